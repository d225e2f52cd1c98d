// Host-side launch interface of the libabm kernels (internal to libabm).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---- K1: plain per-step persistent kernel --------------------------------
struct PlainArgs {
    const double* b;     // weights b_k, k < N
    const double* a;     // weights a_k
    const double* c;     // weights c_k
    const double* gam;   // Gamma(alpha+1), Gamma(alpha+2)
    double alpha, h;
    double x0[4];
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
};
int plain_max_local_chunks(int d);
int plain_chunk();
int plain_part_doubles(int G);
hipError_t launch_plain(const PlainArgs& A, int rhs, hipStream_t st);

// ---- K2: far-field products of the blocked method ------------------------
struct FarArgs {
    const double* b;       // weight tables (padded past N by at least L)
    const double* a;
    const float* b32;      // float copies (far_prec fp32)
    const float* a32;
    const uint16_t* bh[3]; // bf16 split terms (far_prec bf16x3 / bf16x6)
    const uint16_t* ah[3];
    const double* F;       // time-major double history [k][ldF]
    const float* F32;      // time-major float history [k][ldF]
    const uint16_t* Fh[3]; // bf16 split terms of the history, k-blocked (kblocked_index)
    int64_t ldF;
    int64_t mL;            // first history index of the block, m*L
    int64_t kfar;          // far field covers k = 1..kfar (multiple of L)
    int32_t kchunk;        // history rows per chunk (multiple of 512)
    int32_t nchunks;       // ceil(kfar / kchunk)
    int32_t chunks_per_split;
    int32_t nsplit;        // workgroups along the history = partial slices written
    double* part;          // [nsplit][ldP][2L]
    int64_t ldP;           // columns (multiple of the tile width)
};
int far_tile_cols(int L, int prec);
int far_stage_rows();
size_t far_lds_bytes(int L, int kchunk, int prec);
hipError_t launch_far(const FarArgs& A, int L, int prec, hipStream_t st);
size_t far_lp_lds_bytes(int L, int kchunk, int prec);
hipError_t launch_far_lp(const FarArgs& A, int L, int prec, hipStream_t st);
// Chunks of the far range 1..kfar and their grouping into at most max_split
// workgroup ranges; returns the number of partial slices.
int far_split_plan(int64_t kfar, int kchunk, int max_split, int* nchunks, int* chunks_per_split);
hipError_t allow_lds(const void* fn, size_t bytes);   // dynamic LDS above 64 KiB

// ---- K3: near band + predictor/corrector chain ---------------------------
struct TrajDesc {
    double x0[4];
    double p[8];
    double h;
    int64_t N;
    int64_t out_stride;
    double* y_out;
    int32_t col0;          // first column of this trajectory in its group's history
    int32_t pad_;
};
struct ChainArgs {
    const TrajDesc* traj;  // device array, ntraj entries
    int32_t ntraj;
    int32_t nchunks;       // far-field partial slices of this block (0 when m = 0)
    const double* b;
    const double* a;
    const double* c;
    const double* gam;
    double alpha;
    double* F;             // double history [k][ldF]
    float* F32;            // float copy (or null)
    uint16_t* Fhi;         // bf16 split terms (or null): hi, second, third
    uint16_t* Fmid;
    uint16_t* Flo;
    int64_t ldF;
    const double* part;    // far partials [nchunks][ldP][2L]
    int64_t ldP;
    int64_t mL;
    double* accn;          // [ntraj][2][d][L] sums carried into the next block
    uint32_t* status;
};
hipError_t launch_chain(const ChainArgs& A, int rhs, int L, hipStream_t st);
hipError_t launch_chain_init(const ChainArgs& A, int rhs, hipStream_t st);

// ---- utilities -----------------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);

}  // namespace abm
