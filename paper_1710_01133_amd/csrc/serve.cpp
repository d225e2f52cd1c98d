// Serving loop of libabm: abm_submit / abm_poll / abm_cancel.
//
// A server thread per context owns two HIP streams and a device arena.
// Requests queue in arrival order; the head of the queue is admitted as soon
// as its device footprint (weight tables, history and its reduced copy,
// carried sums, far partials) fits the free arena memory, so admission is
// FIFO and never over-commits the arena.  Every admitted request is a group
// of one trajectory with its own weight tables (one per distinct order of
// its components).  The server advances all
// admitted requests in ticks, exactly like abm_solve_batch: one far-field
// launch per precision class and one chain launch per right-hand side per
// tick cover every active request, whatever its alpha, N or start time;
// requests admitted while others run join at the next tick (continuous
// batching).  A request's arithmetic does not depend on what else is running
// (each group has its own columns and chunking), so its result is the same
// alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "abm.h"
#include "abm_kernels.h"
#include "abm_runtime.h"

namespace abm {

namespace {

constexpr int kMaxActive = 1024;     // group slots on the device
constexpr int kMaxFar = 4 * kMaxActive;   // far items per tick (one per component at most)
constexpr int kRing = 8;             // ticks in flight (item staging ring)
// one ring slot: a tick's far, chain and init items, packed in that order
constexpr size_t kSlotBytes = kMaxFar * sizeof(FarItem) + 2 * kMaxActive * sizeof(ChainItem);
static_assert(sizeof(FarItem) % alignof(ChainItem) == 0, "packed item staging");
constexpr size_t kAlign = 256;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum ReqState { kQueued, kRunning, kDone };

struct Request {
    uint64_t ticket = 0;
    abm_problem prob{};
    double* y_out = nullptr;
    double t_submit = 0, t_start = 0, t_done = 0;
    ReqState state = kQueued;
    abm_status status = ABM_OK;
    bool cancel = false;
    // device side (valid while running)
    size_t off = 0, bytes = 0;        // arena chunk
    int slot = -1;
    WeightTable W[4] = {};            // one per distinct order
    Group g{};
    int64_t m = 0, nblocks = 0;
    bool finishing = false;           // last work enqueued; waiting for done_ev
    bool cancel_seen = false;         // cancellation observed by the server thread
    hipEvent_t done_ev = nullptr;
    double* final_host = nullptr;     // pinned: last state (4 doubles), the descriptor, then
                                      // the request's device status word (final_status)
    double max_abs_y = 0;
};

// Pinned staging of one request: its final state, the descriptor it uploads
// and the copy of its status word read at completion.
constexpr size_t kFinalHostBytes = 4 * sizeof(double) + sizeof(TrajDesc) + sizeof(uint64_t);
uint32_t* final_status(Request* r)
{
    return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(r->final_host) + 4 * sizeof(double) +
                                       sizeof(TrajDesc));
}

}  // namespace

// most far partial slices per request and block (ABM_SERVE_MAX_SPLIT
// overrides); a slice takes at least 8 history chunks, so a request of up to
// 262144 steps never needs more
int serve_max_split() { return std::max(1, std::min(256, env_int("ABM_SERVE_MAX_SPLIT", 32))); }

struct ServeState {
    abm_ctx* ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    bool started = false;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    // owned by the server thread
    int L = 256, kchunk = 2048, max_split = serve_max_split();
    char* arena = nullptr;
    size_t arena_cap = 0;
    std::map<size_t, size_t> free_list;   // offset -> size
    std::vector<Request*> active;
    std::vector<int> free_slots;
    hipStream_t s0 = nullptr, s1 = nullptr;
    GroupDev* groups_dev = nullptr;
    GroupDev* groups_host = nullptr;      // pinned staging, one entry per slot
    char* stage_dev = nullptr;            // [kRing][kSlotBytes] items of a tick
    char* stage_host = nullptr;           // pinned, the same
    hipEvent_t ring_ev[kRing] = {};
    bool ring_live[kRing] = {};
    int64_t tick = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    uint32_t* status = nullptr;
    std::string error;
};

namespace {

bool arena_alloc(ServeState* S, size_t bytes, size_t* off)
{
    for (auto it = S->free_list.begin(); it != S->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            S->free_list.erase(it);
            if (rest) S->free_list[roff] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(ServeState* S, size_t off, size_t bytes)
{
    auto it = S->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != S->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        S->free_list.erase(nx);
    }
    if (it != S->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            S->free_list.erase(it);
        }
    }
}

// Layout of one request's arena chunk (all offsets 256-byte aligned).
struct TableLayout {
    double alpha;
    size_t gam, b, a, c, b32, a32, bh[3], ah[3];
};
struct ReqLayout {
    TableLayout tab[4];
    int ntab;
    int tab_of[4];                    // table of each component
    size_t F, F32, Fh[3], Fsc, Fq[3], Fqs, traj, accn, part, status, total;
    int64_t wn, rows, ldF, ldC;
    size_t part_half;
    bool narrow, per_comp;
};

ReqLayout layout_of(const abm_problem& p, int L, int kchunk, int max_split)
{
    ReqLayout r{};
    r.wn = p.N + kWeightPad;
    r.rows = p.N + 1 + L;
    r.narrow = env_int("ABM_NARROW", 1) != 0 && hankel_fits(p.far_prec, p.d, L);
    r.per_comp = orders_differ(p);
    {
        Group g{};                    // the column layout of a one-member group
        g.members = {0};
        g.d = p.d;
        g.prec = p.far_prec;
        g.narrow = r.narrow;
        g.per_comp = r.per_comp;
        group_layout(g, L);
        r.ldF = g.ldF;
        r.ldC = g.ldC;
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align_up(bytes); return at; };
    r.ntab = 0;
    for (int c = 0; c < 4; ++c) {
        const double al = order_of(p, c < p.d ? c : 0);
        int t = 0;
        while (t < r.ntab && r.tab[t].alpha != al) ++t;
        r.tab_of[c] = t;
        if (t < r.ntab) continue;
        TableLayout& T = r.tab[r.ntab++];
        T.alpha = al;
        T.gam = take(2 * sizeof(double));
        T.b = take(r.wn * sizeof(double));
        T.a = take(r.wn * sizeof(double));
        T.c = take(r.wn * sizeof(double));
        T.b32 = T.a32 = 0;
        for (int i = 0; i < 3; ++i) T.bh[i] = T.ah[i] = 0;
        if (p.far_prec == ABM_FAR_FP32 || p.far_prec == ABM_FAR_FP16X3) {
            T.b32 = take(r.wn * sizeof(float));
            T.a32 = take(r.wn * sizeof(float));
        } else if (p.far_prec == ABM_FAR_BF16X3 || p.far_prec == ABM_FAR_BF16X6) {
            for (int i = 0; i < 3; ++i) {
                T.bh[i] = take(r.wn * sizeof(uint16_t));
                T.ah[i] = take(r.wn * sizeof(uint16_t));
            }
        }
    }
    for (int i = 0; i < 3; ++i) r.Fh[i] = 0;
    r.F = take((size_t)r.rows * r.ldF * sizeof(double));
    r.F32 = 0;
    if (p.far_prec == ABM_FAR_FP32) r.F32 = take((size_t)r.rows * r.ldF * sizeof(float));
    r.Fsc = 0;
    if (p.far_prec == ABM_FAR_BF16X3 || p.far_prec == ABM_FAR_BF16X6 ||
        p.far_prec == ABM_FAR_FP16X3) {
        const int terms = p.far_prec == ABM_FAR_BF16X6 ? 3 : 2;
        for (int i = 0; i < terms; ++i)
            r.Fh[i] = take((size_t)((r.rows + 7) / 8) * r.ldF * 8 * sizeof(uint16_t));
        if (p.far_prec == ABM_FAR_FP16X3) r.Fsc = take((size_t)(r.rows / 32 + 1) * r.ldF * sizeof(float));
    }
    for (int i = 0; i < 3; ++i) r.Fq[i] = 0;
    r.Fqs = 0;
    if (p.far_prec == ABM_FAR_I8) {
        for (int i = 0; i < 3; ++i) r.Fq[i] = take((size_t)((r.rows + 15) / 16) * r.ldF * 16);
        r.Fqs = take((size_t)(r.rows / L + 1) * r.ldF * sizeof(double));
    }
    r.traj = take(sizeof(TrajDesc));
    r.accn = take((size_t)2 * p.d * L * sizeof(double));
    const int64_t nblocks = (p.N + L - 1) / L;
    const int64_t kfar_max = nblocks >= 2 ? (nblocks - 2) * L : 0;
    const int nsp = std::max(1, r.narrow ? hankel_split_bound(kfar_max, L, max_split)
                                         : far_split_bound(kfar_max, kchunk, max_split));
    r.part_half = (size_t)nsp * r.ldF * 2 * L;
    r.part = take(2 * r.part_half * sizeof(double));
    r.status = take(sizeof(uint32_t));
    r.total = o;
    return r;
}

hipEvent_t pooled_event(ServeState* S)
{
    // events are recycled round-robin; a pool much larger than the ticks in
    // flight guarantees an event is never re-recorded while still awaited
    if (S->ev_pool.empty()) return nullptr;
    hipEvent_t ev = S->ev_pool[S->ev_next];
    S->ev_next = (S->ev_next + 1) % S->ev_pool.size();
    return ev;
}

// Block length and history chunk of the serving loop, the same for every
// request (so a request's sums do not depend on what it is batched with).
abm_status serve_params(int* L, int* kchunk)
{
    *L = env_int("ABM_SERVE_BLOCK_L", 256);
    if (*L != 128 && *L != 256 && *L != 512)
        return fail(ABM_EINVAL, "ABM_SERVE_BLOCK_L must be 128, 256 or 512");
    *kchunk = 2048;
    for (int prec : kBlockedPrecs)
        while (*kchunk > 512 && far_lds_bytes(*L, *kchunk, prec) > kMaxLds) *kchunk -= 512;
    return ABM_OK;
}

abm_status server_init(ServeState* S)
{
    abm_ctx* ctx = S->ctx;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    abm_status ps = serve_params(&S->L, &S->kchunk);
    if (ps) return ps;
    S->arena_cap = ctx->arena_bytes;
    if ((e = hipMalloc((void**)&S->arena, S->arena_cap)) != hipSuccess) return hip_fail(e, "arena");
    S->free_list[0] = S->arena_cap;
    if ((e = hipStreamCreateWithFlags(&S->s0, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&S->s1, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "server streams");

    abm_status s;
    if ((s = dev_alloc((void**)&S->groups_dev, kMaxActive * sizeof(GroupDev), "group slots")) ||
        (s = dev_alloc((void**)&S->stage_dev, (size_t)kRing * kSlotBytes, "item ring")) ||
        (s = dev_alloc((void**)&S->status, sizeof(uint32_t), "status")))
        return s;
    if ((e = hipHostMalloc((void**)&S->groups_host, kMaxActive * sizeof(GroupDev), hipHostMallocDefault)) ||
        (e = hipHostMalloc((void**)&S->stage_host, (size_t)kRing * kSlotBytes, hipHostMallocDefault)))
        return hip_fail(e, "pinned staging");
    for (int i = 0; i < kRing; ++i)
        if ((e = hipEventCreateWithFlags(&S->ring_ev[i], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event");
    S->ev_pool.resize(64 * kRing);
    for (auto& ev : S->ev_pool)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event");
    for (int i = kMaxActive - 1; i >= 0; --i) S->free_slots.push_back(i);
    (void)launch_fill_u32(S->status, 0, 1, S->s0);
    return ABM_OK;
}

// Device setup of an admitted request on stream s0: carve its arena chunk,
// generate its weight tables, publish its group slot and descriptor.
abm_status admit(ServeState* S, Request* r, size_t off, const ReqLayout& lay)
{
    const abm_problem& p = r->prob;
    char* base = S->arena + off;
    r->off = off;
    r->bytes = lay.total;
    r->slot = S->free_slots.back();
    S->free_slots.pop_back();
    for (int t = 0; t < lay.ntab; ++t) {
        const TableLayout& T = lay.tab[t];
        WeightTable& W = r->W[t];
        W.alpha = T.alpha;
        W.n = p.N;
        W.gam = (double*)(base + T.gam);
        W.b = (double*)(base + T.b);
        W.a = (double*)(base + T.a);
        W.c = (double*)(base + T.c);
        W.b32 = T.b32 ? (float*)(base + T.b32) : nullptr;
        W.a32 = T.a32 ? (float*)(base + T.a32) : nullptr;
        for (int i = 0; i < 3; ++i) {
            W.bh[i] = T.bh[i] ? (uint16_t*)(base + T.bh[i]) : nullptr;
            W.ah[i] = T.ah[i] ? (uint16_t*)(base + T.ah[i]) : nullptr;
        }
    }
    Group& g = r->g;
    for (int c = 0; c < 4; ++c) g.table[c] = lay.tab_of[c];
    g.per_comp = lay.per_comp;
    g.deriv = deriv_mask(p);
    g.rhs = p.rhs;
    g.d = p.d;
    g.prec = p.far_prec;
    g.nmax = p.N;
    g.members = {0};
    g.narrow = lay.narrow;
    group_layout(g, S->L);
    if (g.ldF != lay.ldF || g.ldC != lay.ldC) return fail(ABM_EDEVICE, "internal: request layout");
    g.rows = lay.rows;
    g.F = (double*)(base + lay.F);
    g.F32 = lay.F32 ? (float*)(base + lay.F32) : nullptr;
    for (int i = 0; i < 3; ++i) g.Fh[i] = lay.Fh[i] ? (uint16_t*)(base + lay.Fh[i]) : nullptr;
    g.Fsc = lay.Fsc ? (float*)(base + lay.Fsc) : nullptr;
    for (int i = 0; i < 3; ++i) g.Fq[i] = lay.Fq[i] ? (int8_t*)(base + lay.Fq[i]) : nullptr;
    g.Fqs = lay.Fqs ? (double*)(base + lay.Fqs) : nullptr;
    g.traj_dev = (TrajDesc*)(base + lay.traj);
    g.accn = (double*)(base + lay.accn);
    g.part_half = lay.part_half;
    g.nsplit_cap = (int)(lay.part_half / ((size_t)lay.ldF * 2 * S->L));
    g.part[0] = (double*)(base + lay.part);
    g.part[1] = g.part[0] + lay.part_half;
    g.status = (uint32_t*)(base + lay.status);
    r->m = 0;
    r->nblocks = (p.N + S->L - 1) / S->L;

    hipError_t e = launch_fill_u32(g.status, 0, 1, S->s0);
    for (int t = 0; t < lay.ntab && e == hipSuccess; ++t) {
        WeightTable& W = r->W[t];
        e = launch_weights(W.alpha, lay.wn, W.gam, W.b, W.a, W.c, S->s0);
        if (e == hipSuccess && (W.b32 || W.bh[0]))
            e = launch_weights_lowp(lay.wn, W.b, W.a, W.b32, W.a32, W.bh, W.ah, S->s0);
    }
    if (e != hipSuccess) return hip_fail(e, "request weights");
    // descriptor and group slot through pinned staging (the slot's staging
    // entry is only rewritten when the slot is reused, long after this copy)
    if ((e = hipHostMalloc((void**)&r->final_host, kFinalHostBytes, hipHostMallocDefault)) !=
        hipSuccess)
        return hip_fail(e, "pinned staging");
    const WeightTable* Wc[4];
    for (int c = 0; c < 4; ++c) Wc[c] = &r->W[lay.tab_of[c]];
    GroupDev gd = group_dev(g, Wc);
    S->groups_host[r->slot] = gd;
    if ((e = hipMemcpyAsync(&S->groups_dev[r->slot], &S->groups_host[r->slot], sizeof(GroupDev),
                            hipMemcpyHostToDevice, S->s0)) != hipSuccess)
        return hip_fail(e, "slot upload");
    TrajDesc& T = *reinterpret_cast<TrajDesc*>(r->final_host + 4);
    memset(&T, 0, sizeof T);
    for (int i = 0; i < 4; ++i) {
        T.x0[i] = p.x0[i];
        T.x1[i] = p.x1[i];
    }
    for (int i = 0; i < 8; ++i) T.p[i] = p.p[i];
    T.h = p.h;
    T.N = p.N;
    T.out_stride = p.out_stride;
    T.y_out = r->y_out;
    T.col0 = g.col0[0];
    T.cstride = (int32_t)g.ldC;
    if ((e = hipMemcpyAsync(g.traj_dev, &T, sizeof T, hipMemcpyHostToDevice, S->s0)) != hipSuccess)
        return hip_fail(e, "descriptor upload");
    if ((e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "event");
    return ABM_OK;
}

void release(ServeState* S, Request* r)
{
    arena_free(S, r->off, r->bytes);
    if (r->slot >= 0) S->free_slots.push_back(r->slot);
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    if (r->final_host) (void)hipHostFree(r->final_host);
    r->done_ev = nullptr;
    r->final_host = nullptr;
    r->slot = -1;
}

// Enqueue one tick for every active request.
abm_status enqueue_tick(ServeState* S, const std::vector<Request*>& fresh)
{
    const int ring = (int)(S->tick % kRing);
    hipError_t e;
    if (S->ring_live[ring] && (e = hipEventSynchronize(S->ring_ev[ring])) != hipSuccess)
        return hip_fail(e, "ring wait");
    // items grouped by class: far by launch class, chain by kind, init by rhs
    std::vector<FarItem> far[kFarClasses];
    std::vector<ChainItem> chain[kChainKinds], init[kRhsCount];
    for (Request* r : S->active) {
        if (r->finishing || r->cancel_seen) continue;
        const std::vector<int64_t> memberN{r->prob.N};
        const int cls = far_class(r->g.prec, r->g.narrow);
        const int kind = chain_kind(r->g.rhs, r->g.per_comp);
        const size_t f0 = far[cls].size(), c0 = chain[kind].size();
        block_items(r->g, r->slot, r->m, S->L, S->kchunk, S->max_split, memberN,
                    &far[cls], &chain[kind]);
        // every item must fit the request's partial buffers (checked, not assumed)
        for (size_t k = f0; k < far[cls].size(); ++k) {
            const FarItem& it = far[cls][k];
            if (it.nsplit > r->g.nsplit_cap || it.ldP > r->g.ldF ||
                it.coff + (int64_t)it.ncols > r->g.ldF ||
                (r->g.narrow && !hankel_fits(r->g.prec, it.ncols, S->L)))
                return fail(ABM_EDEVICE, "internal: far item exceeds a request's partial buffer");
        }
        for (size_t k = c0; k < chain[kind].size(); ++k) {
            if (chain[kind][k].nsplit > r->g.nsplit_cap)
                return fail(ABM_EDEVICE, "internal: chain item exceeds a request's partial buffer");
            // a narrow request's slices are summed into the first one after
            // its far field (launch_far_reduce)
            if (r->g.narrow) chain[kind][k].nsplit = std::min(chain[kind][k].nsplit, 1);
        }
    }
    for (Request* r : fresh) {
        ChainItem c{};
        c.group = r->slot;
        c.member = 0;
        init[r->g.rhs].push_back(c);
    }
    int nf = 0, nc = 0, ni = 0;
    size_t nfar = 0, nchain = 0;
    for (const auto& v : far) nfar += v.size();
    for (const auto& v : chain) nchain += v.size();
    size_t ninit = 0;
    for (const auto& v : init) ninit += v.size();
    if (nfar > (size_t)kMaxFar || nchain > (size_t)kMaxActive || ninit > (size_t)kMaxActive)
        return fail(ABM_EDEVICE, "internal: more items than the staging ring holds");
    // the slot holds far, chain and init items back to back, uploaded by one copy
    char* hb = S->stage_host + (size_t)ring * kSlotBytes;
    char* db = S->stage_dev + (size_t)ring * kSlotBytes;
    const size_t off_c = nfar * sizeof(FarItem), off_i = off_c + nchain * sizeof(ChainItem);
    const size_t used = off_i + ninit * sizeof(ChainItem);
    FarItem* fh = reinterpret_cast<FarItem*>(hb);
    ChainItem* ch = reinterpret_cast<ChainItem*>(hb + off_c);
    ChainItem* ih = reinterpret_cast<ChainItem*>(hb + off_i);
    Span fsp[kFarClasses], csp[kChainKinds], isp[kRhsCount];
    for (int k = 0; k < kFarClasses; ++k) {
        fsp[k].offset = nf;
        fsp[k].count = (int32_t)far[k].size();
        for (const FarItem& it : far[k]) {
            fsp[k].max_x = std::max(fsp[k].max_x, it.ncoltiles);
            fsp[k].max_y = std::max(fsp[k].max_y, it.nsplit);
            fsp[k].max_cols = std::max(fsp[k].max_cols, it.ncols);
            fh[nf++] = it;
        }
    }
    for (int k = 0; k < kChainKinds; ++k) {
        csp[k].offset = nc;
        csp[k].count = (int32_t)chain[k].size();
        for (const ChainItem& it : chain[k]) ch[nc++] = it;
    }
    for (int k = 0; k < kRhsCount; ++k) {
        isp[k].offset = ni;
        isp[k].count = (int32_t)init[k].size();
        for (const ChainItem& it : init[k]) ih[ni++] = it;
    }
    FarItem* fd = reinterpret_cast<FarItem*>(db);
    ChainItem* cd = reinterpret_cast<ChainItem*>(db + off_c);
    ChainItem* id = reinterpret_cast<ChainItem*>(db + off_i);
    // The two streams swap roles every tick (as in the batched path): the
    // chains of tick t run on sc = S[t mod 2]; the item uploads and the far
    // field of the next blocks go to the other stream sf, after the chains of
    // tick t-1 (the far field's input) in stream order.  The chains wait for
    // one event on sf recorded after the uploads, which also covers the
    // previous chains and any admission set-up enqueued on sf; the far field
    // of their own blocks, launched a tick earlier, precedes them on sc.
    hipStream_t sc = (S->tick & 1) ? S->s1 : S->s0;
    hipStream_t sf = (S->tick & 1) ? S->s0 : S->s1;
    if (used && (e = hipMemcpyAsync(db, hb, used, hipMemcpyHostToDevice, sf)))
        return hip_fail(e, "item upload");
    hipEvent_t up = pooled_event(S);
    if ((e = hipEventRecord(up, sf)) != hipSuccess) return hip_fail(e, "event");
    for (int k = 0; k < kFarClasses; ++k) {
        if (!fsp[k].count) continue;
        e = launch_far(S->groups_dev, fd + fsp[k].offset, fsp[k].count, fsp[k].max_x, fsp[k].max_y,
                       S->kchunk, S->L, k, sf);
        if (e != hipSuccess) return hip_fail(e, "far-field launch");
        if (is_narrow_class(k) && fsp[k].max_y > 1 &&
            (e = launch_far_reduce(S->groups_dev, fd + fsp[k].offset, fsp[k].count, fsp[k].max_cols,
                                   S->L, sf)) != hipSuccess)
            return hip_fail(e, "partial reduction launch");
    }
    if ((e = hipStreamWaitEvent(sc, up, 0)) != hipSuccess) return hip_fail(e, "wait");
    for (int k = 0; k < kRhsCount; ++k) {
        if (isp[k].count &&
            (e = launch_chain_init(S->groups_dev, id + isp[k].offset, isp[k].count, k, sc)) != hipSuccess)
            return hip_fail(e, "init launch");
    }
    // chains of every kind: one launch (one kernel switching per wave when
    // the tick mixes systems), so they run side by side
    int nkind = 0, nw = 1;
    for (int k = 0; k < kChainKinds; ++k)
        if (csp[k].count) {
            ++nkind;
            nw = std::max(nw, chain_tables(k));
        }
    if (nkind > 1) {
        if ((e = launch_chain_mixed(S->groups_dev, cd, nc, S->L, nw, S->status, sc)) != hipSuccess)
            return hip_fail(e, "chain launch");
    } else {
        for (int k = 0; k < kChainKinds; ++k) {
            if (csp[k].count &&
                (e = launch_chain(S->groups_dev, cd + csp[k].offset, csp[k].count, k, S->L, false, S->status,
                                  sc)) != hipSuccess)
                return hip_fail(e, "chain launch");
        }
    }
    // requests whose last block ran in this tick: copy the last state, mark done
    for (Request* r : S->active) {
        if (r->finishing) continue;
        if (r->cancel_seen) {
            // no more work for it; done once what was already issued has run
            if ((e = hipEventRecord(r->done_ev, sc)) != hipSuccess) return hip_fail(e, "event");
            r->finishing = true;
            continue;
        }
        r->m += 1;
        if (r->m >= r->nblocks) {
            const int64_t nout = n_out(r->prob.N, r->prob.out_stride);
            if ((e = hipMemcpyAsync(r->final_host, r->y_out + (nout - 1) * r->prob.d,
                                    r->prob.d * sizeof(double), hipMemcpyDeviceToHost, sc)) ||
                (e = hipMemcpyAsync(final_status(r), r->g.status, sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, sc)))
                return hip_fail(e, "result copy");
            if ((e = hipEventRecord(r->done_ev, sc)) != hipSuccess) return hip_fail(e, "event");
            r->finishing = true;
        }
    }
    if ((e = hipEventRecord(S->ring_ev[ring], sc)) != hipSuccess) return hip_fail(e, "event");
    S->ring_live[ring] = true;
    ++S->tick;
    return ABM_OK;
}

// Fail every queued and running request (the server stops after a device
// error).  Called with S->mu held.  The requests stay owned by S->all until
// polled; pending and active are emptied so that nothing else refers to them.
void fail_all(ServeState* S)
{
    const double t = now_s();
    for (auto& kv : S->all) {
        Request* r = kv.second;
        if (r->state == kDone) continue;
        r->state = kDone;
        r->status = ABM_EDEVICE;
        r->t_done = t;
    }
    S->pending.clear();
    S->active.clear();
    S->stop = true;
}

void server_loop(ServeState* S)
{
    if (server_init(S) != ABM_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->error = abm_last_error();
        fail_all(S);
        return;
    }
    for (;;) {
        std::vector<Request*> fresh;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->active.empty() && S->pending.empty() && !S->stop)
                S->cv.wait_for(lk, std::chrono::milliseconds(50));
            if (S->stop && S->active.empty()) break;
            for (Request* r : S->active) r->cancel_seen = r->cancel_seen || r->cancel;
            // FIFO admission by arena memory and slots
            while (!S->pending.empty() && !S->free_slots.empty() &&
                   (int)S->active.size() < kMaxActive) {
                Request* r = S->pending.front();
                if (r->cancel) {
                    S->pending.pop_front();
                    r->state = kDone;
                    r->status = ABM_ECANCELED;
                    r->t_done = now_s();
                    continue;
                }
                const ReqLayout lay = layout_of(r->prob, S->L, S->kchunk, S->max_split);
                if (lay.total > S->arena_cap) {   // can never fit: fail it, keep the queue moving
                    S->pending.pop_front();
                    r->state = kDone;
                    r->status = ABM_ENOMEM;
                    r->t_done = now_s();
                    continue;
                }
                size_t off = 0;
                if (!arena_alloc(S, lay.total, &off)) break;   // head waits for memory
                S->pending.pop_front();
                if (admit(S, r, off, lay) != ABM_OK) {
                    // whatever admission enqueued has run before its memory,
                    // slot, event and staging are given back
                    (void)hipStreamSynchronize(S->s0);
                    release(S, r);
                    r->state = kDone;
                    r->status = ABM_EDEVICE;
                    r->t_done = now_s();
                    continue;
                }
                r->state = kRunning;
                r->t_start = now_s();
                S->active.push_back(r);
                fresh.push_back(r);
            }
        }
        bool any_work = false;
        for (Request* r : S->active)
            if (!r->finishing) any_work = true;   // includes a cancel to retire
        if (any_work && enqueue_tick(S, fresh) != ABM_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->error = abm_last_error();
            fail_all(S);
            break;
        }
        // completions
        std::vector<Request*> keep;
        for (Request* r : S->active) {
            if (r->finishing && hipEventQuery(r->done_ev) == hipSuccess) {
                const double t = now_s();
                double mx = 0;
                // the chains raised the request's own status word if any of
                // its states became non-finite
                bool bad = !r->cancel_seen && *final_status(r) != 0;
                for (int i = 0; i < r->prob.d && !r->cancel_seen; ++i) {
                    bad |= !std::isfinite(r->final_host[i]);
                    mx = std::max(mx, std::fabs(r->final_host[i]));
                }
                release(S, r);
                std::lock_guard<std::mutex> lk(S->mu);
                r->max_abs_y = mx;
                r->status = r->cancel_seen ? ABM_ECANCELED : (bad ? ABM_EDEVICE : ABM_OK);
                r->state = kDone;
                r->t_done = t;
            } else {
                keep.push_back(r);
            }
        }
        S->active.swap(keep);
        if (!any_work && !S->active.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    (void)hipStreamSynchronize(S->s0);
    (void)hipStreamSynchronize(S->s1);

}

}  // namespace

abm_status serve_create(abm_ctx* ctx)
{
    ServeState* S = new (std::nothrow) ServeState();
    if (!S) return fail(ABM_ENOMEM, "server state");
    S->ctx = ctx;
    ctx->serve = S;
    return ABM_OK;
}

void serve_shutdown(abm_ctx* ctx)
{
    ServeState* S = ctx->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Request* r : S->pending) {
            r->cancel = true;
        }
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    // every request not yet polled is in S->all (and only there once the
    // thread has ended: pending and active hold a subset of it)
    S->pending.clear();
    S->active.clear();
    for (auto& kv : S->all) {
        if (kv.second->final_host) (void)hipHostFree(kv.second->final_host);
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        delete kv.second;
    }
    S->all.clear();
    if (S->arena) (void)hipFree(S->arena);
    dev_free(S->groups_dev);
    dev_free(S->stage_dev);
    dev_free(S->status);
    if (S->groups_host) (void)hipHostFree(S->groups_host);
    if (S->stage_host) (void)hipHostFree(S->stage_host);
    for (auto ev : S->ring_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : S->ev_pool) (void)hipEventDestroy(ev);
    if (S->s0) (void)hipStreamDestroy(S->s0);
    if (S->s1) (void)hipStreamDestroy(S->s1);

    delete S;
    ctx->serve = nullptr;
}

}  // namespace abm

using namespace abm;

extern "C" {

abm_status abm_submit(abm_ctx* ctx, const abm_problem* prob, double* y_out, uint64_t* ticket)
{
    if (!ctx || !prob || !y_out || !ticket) return fail(ABM_EINVAL, "NULL argument");
    abm_status s = validate(*prob, 0);
    if (s) return s;
    if (prob->far_prec == ABM_FAR_DD)
        return fail(ABM_EINVAL, "double-double (ABM_FAR_DD) runs on abm_solve only");
    ServeState* S = ctx->serve;   // made with the context, fixed until it is destroyed
    int L = 0, kchunk = 0;
    if ((s = serve_params(&L, &kchunk))) return s;
    if (prob->far_prec == ABM_FAR_I8 && L > 256)
        return fail(ABM_EINVAL, "the int8 far field needs block length 128 or 256 (ABM_SERVE_BLOCK_L=%d)", L);
    const ReqLayout lay = layout_of(*prob, L, kchunk, S->max_split);
    if (lay.total > ctx->arena_bytes)
        return fail(ABM_ENOMEM, "request needs %zu bytes, the arena has %zu", lay.total,
                    ctx->arena_bytes);
    Request* r = new Request();
    r->prob = *prob;
    r->y_out = y_out;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete r;
            return fail(ABM_EDEVICE, "server stopped: %s", S->error.c_str());
        }
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->pending.push_back(r);
        if (!S->started) {
            S->started = true;
            S->th = std::thread(server_loop, S);
        }
    }
    S->cv.notify_all();
    *ticket = r->ticket;
    return ABM_OK;
}

abm_status abm_request_bytes(abm_ctx* ctx, const abm_problem* prob, size_t* bytes)
{
    if (!ctx || !prob || !bytes) return fail(ABM_EINVAL, "NULL argument");
    abm_status s = validate(*prob, 0);
    if (s) return s;
    if (prob->far_prec == ABM_FAR_DD)
        return fail(ABM_EINVAL, "double-double (ABM_FAR_DD) is not served");
    int L = 0, kchunk = 0;
    if ((s = serve_params(&L, &kchunk))) return s;
    if (prob->far_prec == ABM_FAR_I8 && L > 256)
        return fail(ABM_EINVAL, "the int8 far field needs block length 128 or 256 (ABM_SERVE_BLOCK_L=%d)", L);
    *bytes = layout_of(*prob, L, kchunk, ctx->serve->max_split).total;
    return ABM_OK;
}

abm_status abm_poll(abm_ctx* ctx, uint64_t ticket, abm_result* res)
{
    if (!ctx || !res) return fail(ABM_EINVAL, "NULL argument");
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ABM_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    if (r->state != kDone) return ABM_EAGAIN;
    res->status = r->status;
    res->t_submit = r->t_submit;
    res->t_start = r->t_start;
    res->t_done = r->t_done;
    res->max_abs_y = r->max_abs_y;
    S->all.erase(it);
    delete r;
    return ABM_OK;
}

abm_status abm_cancel(abm_ctx* ctx, uint64_t ticket)
{
    if (!ctx) return fail(ABM_EINVAL, "NULL argument");
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ABM_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    it->second->cancel = true;
    return ABM_OK;
}

}  // extern "C"
