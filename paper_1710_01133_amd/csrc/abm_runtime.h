// Internal runtime structures of libabm (contexts, plans, groups).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>
#include <vector>

#include "abm.h"
#include "abm_kernels.h"

namespace abm {

constexpr int64_t kMaxSteps = (int64_t)1 << 30;   // step counters are 32-bit on the device
constexpr int64_t kWeightPad = 2048;                // weight tables extend this far past N
constexpr int kPlainDefaultG = 128;
constexpr size_t kMaxLds = 160 * 1024;              // LDS of one gfx950 CU
constexpr uint32_t kSpinLimit = 1u << 22;           // a few seconds of polling (each poll is a memory round trip)

struct ServeState;

struct WeightTable {
    double alpha;
    int64_t n;        // longest N using the table
    double* gam;      // Gamma(alpha+1), Gamma(alpha+2)
    double* b;        // n + kWeightPad doubles each
    double* a;
    double* c;
    // reduced copies for the far field (allocated on demand)
    float* b32;
    float* a32;
    uint16_t* bh[3];  // bf16 split terms of b
    uint16_t* ah[3];
};

// Trajectories sharing one weight table, one right-hand side and one far-field
// precision: their components form the columns of one time-major history.
struct Group {
    int table;
    int rhs;
    int d;
    int prec;
    int64_t nmax;                 // longest trajectory
    std::vector<int> members;     // problem indices, N descending
    std::vector<int32_t> col0;    // first column of each member
    std::vector<int64_t> active_cols;   // per block m: columns of members with N > mL
    std::vector<int32_t> active_traj;   // per block m: members with N > mL
    int64_t cols;                 // real columns
    int64_t ldF;                  // padded columns
    int64_t rows;                 // history rows allocated
    double* F;
    float* F32;
    uint16_t* Fh[3];
    TrajDesc* traj_dev;           // members' descriptors (device)
    double* accn;                 // sums carried into the next block [member][2][d][L]
    TrajDesc* traj_host;          // pinned staging copy of the descriptors
    hipEvent_t traj_ev;           // recorded after the last upload from traj_host
    bool traj_ev_live;
};

}  // namespace abm

struct abm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t arena_bytes = 0;
    int n_cu = 0;
    abm::ServeState* serve = nullptr;
};

struct abm_plan_s {
    abm_ctx* ctx = nullptr;
    int32_t B = 0;
    std::vector<abm_problem> shape;
    std::vector<abm::WeightTable> tables;
    std::vector<int> table_of;
    uint32_t* status = nullptr;
    // plain path (B == 1)
    int plain_G = 0;
    int plain_nloc = 0;
    std::string plain_error;
    double* part = nullptr;
    uint32_t* flags = nullptr;
    // blocked path
    int L = 0;
    int kchunk = 0;
    int max_split = 8;
    std::vector<abm::Group> groups;
    double* ffpart = nullptr;     // far partials, sized for the largest group
    size_t ffpart_bytes = 0;
    // far field on its own stream, overlapping the chain
    bool overlap = true;
    hipStream_t far_stream = nullptr;
    std::vector<hipEvent_t> sync_events;
    // optional per-launch timing
    bool timing = false;
    std::vector<hipEvent_t> events;
};

namespace abm {

abm_status fail(abm_status code, const char* fmt, ...);
abm_status hip_fail(hipError_t e, const char* what);
int rhs_dim(int rhs);
int64_t n_out(int64_t N, int64_t stride);
abm_status validate(const abm_problem& p, int idx);
int env_int(const char* name, int dflt);
abm_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p);

abm_status plain_setup(abm_plan_s* pl);
abm_status batch_setup(abm_plan_s* pl);
void batch_teardown(abm_plan_s* pl);
void free_reduced(WeightTable& t);
void serve_shutdown(abm_ctx* ctx);

}  // namespace abm
