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

// Trajectories sharing their orders (one weight table per component, all the
// same table unless per_comp), one right-hand side and one far-field
// precision: their components form the columns of one time-major history,
// member-major (component i of member j at j*d + i) or, when per_comp,
// component-major (at i*ldC + j) so that every column tile holds one order.
struct Group {
    int table[4] = {0, 0, 0, 0};
    bool per_comp = false;
    int deriv = 0;                // bit i: component i has order above 1
    int64_t ldC = 0;              // per_comp: columns per component block
    int rhs = 0;
    int d = 0;
    int prec = 0;
    int64_t nmax = 0;             // longest trajectory
    std::vector<int> members;     // problem indices, N descending
    std::vector<int32_t> col0;    // first column of each member
    int64_t cols = 0;             // real columns
    int64_t ldF = 0;              // padded columns (narrow groups: real columns)
    bool narrow = false;          // far field by the blocked convolution
    int split_cap = 0;            // narrow groups: most partial slices per block (0: the plan's)
    int64_t rows = 0;             // history rows allocated
    double* F = nullptr;
    float* F32 = nullptr;
    uint16_t* Fh[3] = {nullptr, nullptr, nullptr};
    float* Fsc = nullptr;
    int8_t* Fq[3] = {nullptr, nullptr, nullptr};
    double* Fqs = nullptr;
    TrajDesc* traj_dev = nullptr;   // members' descriptors (device)
    double* accn = nullptr;         // sums carried into the next block [member][2][d][L]
    double* part[2] = {nullptr, nullptr};   // far partials by block parity
    size_t part_half = 0;           // doubles per partial buffer
    int nsplit_cap = 0;             // partial slices each buffer holds
    TrajDesc* traj_host = nullptr;  // pinned staging copy of the descriptors
    hipEvent_t traj_ev = nullptr;   // recorded after the last upload from traj_host
    bool traj_ev_live = false;
    uint32_t* status = nullptr;     // the group's own status word (serving), or null
};

// A run of work items of one launch: offset/count in an item array and the
// grid extents it needs.
struct Span {
    int64_t offset = 0;
    int32_t count = 0;
    int32_t max_x = 0;
    int32_t max_y = 0;
    int32_t max_cols = 0;   // far spans: the widest item (columns)
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
    std::vector<int> table_of;    // [problem][component]: 4 entries per problem
    uint32_t* status = nullptr;
    // plain path (B == 1)
    int plain_G = 0;
    int plain_nloc = 0;
    bool plain_single = false;    // the one-workgroup form (short histories)
    bool dd = false;              // double-double plan (ABM_FAR_DD): plain path only, tables
                                  // of (hi, lo) pairs
    std::string plain_error;
    double* part = nullptr;
    uint32_t* flags = nullptr;
    // blocked path: groups and their static tick schedule
    abm_tuning tune{};            // requested blocking (zero fields: defaults)
    bool allow_narrow = true;
    int L = 0;
    int kchunk = 0;
    int max_split = 8;
    std::vector<abm::Group> groups;
    abm::GroupDev* groups_dev = nullptr;
    abm::FarItem* far_items_dev = nullptr;
    abm::ChainItem* chain_items_dev = nullptr;
    abm::ChainItem* init_items_dev = nullptr;
    int64_t ticks = 0;
    std::vector<abm::Span> far_spans;     // [tick][far launch class]
    std::vector<abm::Span> chain_spans;   // [tick][chain kind]
    std::vector<char> chain_spread;       // [tick]: chains one wave per SIMD (small far field beside)
    std::vector<abm::Span> init_spans;    // [rhs]
    int64_t far_macs = 0;
    // far field on its own stream, overlapping the chain
    bool overlap = true;
    hipStream_t far_stream = nullptr;
    std::vector<hipEvent_t> sync_events;
    // optional per-launch timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    // launch sequence replayed from a graph captured at the first graph solve
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_far_launches = 0;
    int64_t graph_chain_launches = 0;
};

namespace abm {

abm_status fail(abm_status code, const char* fmt, ...);
abm_status hip_fail(hipError_t e, const char* what);
int rhs_dim(int rhs);
int64_t n_out(int64_t N, int64_t stride);
abm_status validate(const abm_problem& p, int idx);
double order_of(const abm_problem& p, int comp);   // order of component comp
bool orders_differ(const abm_problem& p);          // components of different orders
int deriv_mask(const abm_problem& p);              // bit i: component i of order above 1
bool same_orders(const abm_problem& a, const abm_problem& b);
int env_int(const char* name, int dflt);
abm_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p);

// Launch shape of the plain path for one problem: the one-workgroup form, or
// G cooperative workgroups holding nloc history chunks each.
struct PlainShape {
    bool single;
    int G;
    int nloc;
};
// Weight tables of each component (all the same unless orders differ).
struct PlainTables {
    const double* b[4];
    const double* a[4];
    const double* c[4];
    const double* gam[4];
    double alpha[4];
};
abm_status plain_shape(const abm_problem& p, int n_cu, PlainShape* out);
PlainArgs plain_args(const abm_problem& prob, const PlainTables& T, const PlainShape& sh,
                     double* part, uint32_t* flags, uint32_t* status, double* y_out);
// flags reset (cooperative form) and the kernel, on st
hipError_t plain_enqueue(const PlainArgs& A, const PlainShape& sh, int kind, hipStream_t st);
abm_status plain_setup(abm_plan_s* pl);
abm_status plain_setup_dd(abm_plan_s* pl);
abm_status batch_setup(abm_plan_s* pl);
void batch_teardown(abm_plan_s* pl);
void free_reduced(WeightTable& t);
void free_group(Group& g);
abm_status ensure_reduced_weights(WeightTable& W, int prec, hipStream_t st);
abm_status alloc_group(Group& g, int L, int nsplit_max, hipStream_t st);
GroupDev group_dev(const Group& g, const WeightTable* const W[4]);
// Column layout of a group of nm members: ldF, ldC and each member's col0 /
// cstride follow from (per_comp, narrow, d, tile width).
void group_layout(Group& g, int L);
void block_items(const Group& g, int gi, int64_t m, int L, int kchunk, int max_split,
                 const std::vector<int64_t>& memberN, std::vector<FarItem>* far,
                 std::vector<ChainItem>* chain);
int64_t group_far_split_max(const Group& g, int L, int kchunk, int max_split);
abm_status choose_blocking(abm_plan_s* pl, const abm_problem* probs, int B);
abm_status serve_create(abm_ctx* ctx);
void serve_shutdown(abm_ctx* ctx);

}  // namespace abm
