// Blocked batch path: plan-time grouping and sizing, and the per-block launch
// sequence of abm_solve_batch (far-field product, then the chain).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "abm.h"
#include "abm_kernels.h"
#include "abm_runtime.h"

namespace abm {

namespace {

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool valid_L(int L) { return L == 64 || L == 128 || L == 256 || L == 512; }

}  // namespace

void free_reduced(WeightTable& t)
{
    dev_free(t.b32);
    dev_free(t.a32);
    for (int i = 0; i < 3; ++i) {
        dev_free(t.bh[i]);
        dev_free(t.ah[i]);
        t.bh[i] = t.ah[i] = nullptr;
    }
    t.b32 = t.a32 = nullptr;
}

void batch_teardown(abm_plan_s* pl)
{
    for (hipEvent_t ev : pl->events) (void)hipEventDestroy(ev);
    pl->events.clear();
    for (auto& g : pl->groups) {
        dev_free(g.F);
        dev_free(g.F32);
        for (int i = 0; i < 3; ++i) dev_free(g.Fh[i]);
        dev_free(g.traj_dev);
        dev_free(g.accn);
        if (g.traj_host) (void)hipHostFree(g.traj_host);
        if (g.traj_ev) (void)hipEventDestroy(g.traj_ev);
    }
    pl->groups.clear();
    dev_free(pl->ffpart);
    pl->ffpart = nullptr;
    for (hipEvent_t ev : pl->sync_events) (void)hipEventDestroy(ev);
    pl->sync_events.clear();
    if (pl->far_stream) (void)hipStreamDestroy(pl->far_stream);
    pl->far_stream = nullptr;
}

abm_status batch_setup(abm_plan_s* pl)
{
    hipStream_t st = pl->ctx->stream;
    int L = env_int("ABM_BLOCK_L", 256);
    if (!valid_L(L)) return fail(ABM_EINVAL, "ABM_BLOCK_L=%d not in {64,128,256,512}", L);
    int kchunk = env_int("ABM_KCHUNK", 2048);
    if (kchunk < 512 || kchunk % 512)
        return fail(ABM_EINVAL, "ABM_KCHUNK=%d must be a positive multiple of 512", kchunk);
    for (int i = 0; i < pl->B; ++i)
        if (pl->shape[i].far_prec != ABM_FAR_FP64 && L < 128)
            return fail(ABM_EINVAL, "problem %d: reduced-precision far field needs block length >= 128", i);
    // largest chunk whose LDS footprint fits every precision used by the plan
    for (int i = 0; i < pl->B; ++i)
        while (kchunk > 512 && far_lds_bytes(L, kchunk, pl->shape[i].far_prec) > kMaxLds) kchunk -= 512;
    pl->L = L;
    pl->kchunk = kchunk;
    pl->max_split = env_int("ABM_MAX_SPLIT", 8);
    if (pl->max_split < 1) return fail(ABM_EINVAL, "ABM_MAX_SPLIT must be >= 1");

    // groups: (weight table, rhs, precision); members sorted by N descending
    std::map<std::tuple<int, int, int>, int> key_to_group;
    for (int i = 0; i < pl->B; ++i) {
        const abm_problem& p = pl->shape[i];
        auto key = std::make_tuple(pl->table_of[i], p.rhs, p.far_prec);
        auto it = key_to_group.find(key);
        if (it == key_to_group.end()) {
            Group g{};
            g.table = pl->table_of[i];
            g.rhs = p.rhs;
            g.d = p.d;
            g.prec = p.far_prec;
            pl->groups.push_back(g);
            it = key_to_group.emplace(key, (int)pl->groups.size() - 1).first;
        }
        pl->groups[it->second].members.push_back(i);
    }
    size_t ff_need = 0;
    for (auto& g : pl->groups) {
        const int TN = far_tile_cols(L, g.prec);
        std::stable_sort(g.members.begin(), g.members.end(),
                         [&](int x, int y) { return pl->shape[x].N > pl->shape[y].N; });
        g.nmax = pl->shape[g.members[0]].N;
        g.cols = (int64_t)g.members.size() * g.d;
        g.ldF = round_up(g.cols, TN);
        g.rows = g.nmax + 1 + L;
        g.col0.resize(g.members.size());
        for (size_t j = 0; j < g.members.size(); ++j) g.col0[j] = (int32_t)(j * g.d);
        const int64_t nblocks = (g.nmax + L - 1) / L;
        g.active_cols.resize(nblocks);
        g.active_traj.resize(nblocks);
        for (int64_t m = 0; m < nblocks; ++m) {
            int32_t cnt = 0;
            for (int idx : g.members)
                if (pl->shape[idx].N > m * L) ++cnt;
            g.active_traj[m] = cnt;
            g.active_cols[m] = round_up((int64_t)cnt * g.d, TN);
        }
        int nc = 0, cps = 0;
        const int64_t kfar_max = nblocks >= 2 ? (nblocks - 2) * L : 0;   // far(m) covers (m-1)L
        const int64_t nsp = far_split_plan(kfar_max, kchunk, pl->max_split, &nc, &cps);
        ff_need = std::max(ff_need, (size_t)nsp * g.ldF * 2 * L * sizeof(double));
        abm_status s;
        if ((s = dev_alloc((void**)&g.F, (size_t)g.rows * g.ldF * sizeof(double), "history")))
            return s;
        hipError_t e = hipMemsetAsync(g.F, 0, (size_t)g.rows * g.ldF * sizeof(double), st);
        if (e != hipSuccess) return hip_fail(e, "history clear");
        // reduced copies of the history read by the far field
        if (g.prec == ABM_FAR_FP32) {
            const size_t bytes = (size_t)g.rows * g.ldF * sizeof(float);
            if ((s = dev_alloc((void**)&g.F32, bytes, "float history"))) return s;
            if ((e = hipMemsetAsync(g.F32, 0, bytes, st)) != hipSuccess) return hip_fail(e, "clear");
        } else if (g.prec == ABM_FAR_BF16X3 || g.prec == ABM_FAR_BF16X6) {
            const int terms = g.prec == ABM_FAR_BF16X3 ? 2 : 3;
            const size_t bytes = (size_t)((g.rows + 7) / 8) * g.ldF * 8 * sizeof(uint16_t);
            for (int tt = 0; tt < terms; ++tt) {
                if ((s = dev_alloc((void**)&g.Fh[tt], bytes, "bf16 history"))) return s;
                if ((e = hipMemsetAsync(g.Fh[tt], 0, bytes, st)) != hipSuccess) return hip_fail(e, "clear");
            }
        }
        // reduced copies of the weights, once per table
        WeightTable& W = pl->tables[g.table];
        const int64_t wn = W.n + kWeightPad;
        if (g.prec == ABM_FAR_FP32 && !W.b32) {
            if ((s = dev_alloc((void**)&W.b32, wn * sizeof(float), "float weights")) ||
                (s = dev_alloc((void**)&W.a32, wn * sizeof(float), "float weights")))
                return s;
            uint16_t* none[3] = {nullptr, nullptr, nullptr};
            if ((e = launch_weights_lowp(wn, W.b, W.a, W.b32, W.a32, none, none, st)) != hipSuccess)
                return hip_fail(e, "weight conversion");
        }
        if ((g.prec == ABM_FAR_BF16X3 || g.prec == ABM_FAR_BF16X6) && !W.bh[2]) {
            for (int tt = 0; tt < 3; ++tt) {
                if (W.bh[tt]) continue;
                if ((s = dev_alloc((void**)&W.bh[tt], wn * sizeof(uint16_t), "bf16 weights")) ||
                    (s = dev_alloc((void**)&W.ah[tt], wn * sizeof(uint16_t), "bf16 weights")))
                    return s;
            }
            if ((e = launch_weights_lowp(wn, W.b, W.a, nullptr, nullptr, W.bh, W.ah, st)) != hipSuccess)
                return hip_fail(e, "weight conversion");
        }
        if ((s = dev_alloc((void**)&g.traj_dev, g.members.size() * sizeof(TrajDesc), "descriptors")))
            return s;
        if ((s = dev_alloc((void**)&g.accn, g.members.size() * 2 * g.d * L * sizeof(double), "carried sums")))
            return s;
        e = hipHostMalloc((void**)&g.traj_host, g.members.size() * sizeof(TrajDesc), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "pinned descriptors");
        e = hipEventCreateWithFlags(&g.traj_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "event");
    }
    // two partial buffers: the far field of block m+1 is written while the
    // chain of block m reads block m's
    pl->ffpart_bytes = ff_need;
    if (ff_need) {
        abm_status s = dev_alloc((void**)&pl->ffpart, 2 * ff_need, "far partials");
        if (s) return s;
    }
    pl->overlap = env_int("ABM_OVERLAP", 1) != 0;
    if (pl->overlap) {
        hipError_t e = hipStreamCreateWithFlags(&pl->far_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "far stream");
    }
    return ABM_OK;
}

}  // namespace abm

using namespace abm;

extern "C" abm_status abm_solve_batch(abm_plan_t* pl, const abm_problem* probs, int32_t B,
                                      double* const* y_out, abm_stats* stats)
{
    if (!pl || !probs || !y_out) return fail(ABM_EINVAL, "NULL argument");
    if (B != pl->B) return fail(ABM_EINVAL, "B=%d but the plan was made for %d problems", B, pl->B);
    for (int i = 0; i < B; ++i) {
        abm_status s = validate(probs[i], i);
        if (s) return s;
        const abm_problem& a = probs[i];
        const abm_problem& b = pl->shape[i];
        if (a.rhs != b.rhs || a.d != b.d || a.alpha != b.alpha || a.N != b.N ||
            a.far_prec != b.far_prec || a.out_stride != b.out_stride)
            return fail(ABM_EINVAL, "problem %d does not match the plan", i);
        if (!y_out[i]) return fail(ABM_EINVAL, "y_out[%d] is NULL", i);
    }
    hipError_t e = hipSetDevice(pl->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = pl->ctx->stream;
    const int L = pl->L;
    abm_stats S{};
    // event pairs around launches when timing is on: (kind, first, second)
    std::vector<std::pair<int, int>> tev;   // kind 0 far, 1 chain; index of the start event
    size_t ev_used = 0;
    auto ev_next = [&]() -> hipEvent_t {
        if (ev_used == pl->events.size()) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return nullptr;
            pl->events.push_back(ev);
        }
        return pl->events[ev_used++];
    };
    auto timed = [&](int kind, hipStream_t sx, auto&& launch) -> hipError_t {
        if (!pl->timing) return launch();
        hipEvent_t a = ev_next(), b = ev_next();
        if (!a || !b) return hipErrorOutOfMemory;
        const int ia = (int)ev_used - 2;
        hipError_t e1 = hipEventRecord(a, sx);
        if (e1 != hipSuccess) return e1;
        e1 = launch();
        if (e1 != hipSuccess) return e1;
        e1 = hipEventRecord(b, sx);
        tev.push_back({kind, ia});
        return e1;
    };
    // ordering events (no timing), reused across calls
    size_t sync_used = 0;
    auto sync_event = [&]() -> hipEvent_t {
        if (sync_used == pl->sync_events.size()) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
            pl->sync_events.push_back(ev);
        }
        return pl->sync_events[sync_used++];
    };
    S.block_L = L;
    S.n_groups = (int32_t)pl->groups.size();

    for (auto& g : pl->groups) {
        const WeightTable& W = pl->tables[g.table];
        // the staging buffer may still feed the previous solve's upload
        if (g.traj_ev_live) {
            e = hipEventSynchronize(g.traj_ev);
            if (e != hipSuccess) return hip_fail(e, "descriptor staging wait");
        }
        TrajDesc* td = g.traj_host;
        for (size_t j = 0; j < g.members.size(); ++j) {
            const abm_problem& p = probs[g.members[j]];
            TrajDesc& T = td[j];
            memset(&T, 0, sizeof T);
            for (int i = 0; i < 4; ++i) T.x0[i] = p.x0[i];
            for (int i = 0; i < 8; ++i) T.p[i] = p.p[i];
            T.h = p.h;
            T.N = p.N;
            T.out_stride = p.out_stride;
            T.y_out = y_out[g.members[j]];
            T.col0 = g.col0[j];
            S.history_macs += (int64_t)p.d * p.N * (p.N + 1) / 2;
        }
        e = hipMemcpyAsync(g.traj_dev, td, g.members.size() * sizeof(TrajDesc),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        e = hipEventRecord(g.traj_ev, st);
        if (e != hipSuccess) return hip_fail(e, "descriptor event");
        g.traj_ev_live = true;

        ChainArgs C{};
        C.traj = g.traj_dev;
        C.ntraj = (int32_t)g.members.size();
        C.b = W.b;
        C.a = W.a;
        C.c = W.c;
        C.gam = W.gam;
        C.alpha = W.alpha;
        C.F = g.F;
        C.F32 = g.F32;
        C.Fhi = g.Fh[0];
        C.Fmid = g.Fh[1];
        C.Flo = g.Fh[2];
        C.ldF = g.ldF;
        C.part = pl->ffpart;
        C.status = pl->status;
        e = launch_chain_init(C, g.rhs, st);
        if (e != hipSuccess) return hip_fail(e, "chain init launch");

        FarArgs Fa{};
        Fa.b = W.b;
        Fa.a = W.a;
        Fa.b32 = W.b32;
        Fa.a32 = W.a32;
        for (int tt = 0; tt < 3; ++tt) {
            Fa.bh[tt] = W.bh[tt];
            Fa.ah[tt] = W.ah[tt];
            Fa.Fh[tt] = g.Fh[tt];
        }
        Fa.F32 = g.F32;
        Fa.F = g.F;
        Fa.ldF = g.ldF;
        Fa.kchunk = pl->kchunk;
        C.accn = g.accn;

        // far field on s1, chain on s0; far(m+1) overlaps chain(m)
        hipStream_t s1 = pl->overlap ? pl->far_stream : st;
        const int64_t nblocks = (int64_t)g.active_traj.size();
        const size_t ffhalf = pl->ffpart_bytes / sizeof(double);
        hipEvent_t fork = sync_event();
        if (!fork) return fail(ABM_EDEVICE, "event pool");
        if ((e = hipEventRecord(fork, st)) != hipSuccess || (e = hipStreamWaitEvent(s1, fork, 0)) != hipSuccess)
            return hip_fail(e, "stream fork");
        std::vector<hipEvent_t> ev_chain(nblocks, nullptr), ev_far(nblocks + 1, nullptr);
        std::vector<int> nsplit(nblocks + 1, 0);
        for (int64_t m = 0; m < nblocks; ++m) {
            const int64_t mf = m + 1;           // far field of the next block
            if (mf < nblocks && mf >= 2) {
                const int64_t kfar = (mf - 1) * L;
                Fa.mL = mf * L;
                Fa.kfar = kfar;
                Fa.ldP = g.active_cols[mf];
                Fa.nsplit = far_split_plan(kfar, pl->kchunk, pl->max_split, &Fa.nchunks,
                                           &Fa.chunks_per_split);
                Fa.part = pl->ffpart + (mf & 1) * ffhalf;
                nsplit[mf] = Fa.nsplit;
                if ((e = hipStreamWaitEvent(s1, ev_chain[m - 1], 0)) != hipSuccess)
                    return hip_fail(e, "stream wait");
                e = timed(0, s1, [&]() { return launch_far(Fa, L, g.prec, s1); });
                if (e != hipSuccess) return hip_fail(e, "far-field launch");
                ++S.far_launches;
                for (int32_t jj = 0; jj < g.active_traj[mf]; ++jj) {
                    const abm_problem& p = probs[g.members[jj]];
                    const int64_t rows = std::min<int64_t>(L, p.N - mf * L);
                    S.far_macs += (int64_t)p.d * rows * kfar;
                }
                ev_far[mf] = sync_event();
                if (!ev_far[mf] || (e = hipEventRecord(ev_far[mf], s1)) != hipSuccess)
                    return fail(ABM_EDEVICE, "far event");
            }
            if (ev_far[m] && (e = hipStreamWaitEvent(st, ev_far[m], 0)) != hipSuccess)
                return hip_fail(e, "stream wait");
            C.ntraj = g.active_traj[m];
            C.nchunks = nsplit[m];
            C.ldP = g.active_cols[m];
            C.part = pl->ffpart + (m & 1) * ffhalf;
            C.mL = m * L;
            e = timed(1, st, [&]() { return launch_chain(C, g.rhs, L, st); });
            if (e != hipSuccess) return hip_fail(e, "chain launch");
            ++S.chain_launches;
            ev_chain[m] = sync_event();
            if (!ev_chain[m] || (e = hipEventRecord(ev_chain[m], st)) != hipSuccess)
                return fail(ABM_EDEVICE, "chain event");
        }
        hipEvent_t join = sync_event();
        if (!join || (e = hipEventRecord(join, s1)) != hipSuccess ||
            (e = hipStreamWaitEvent(st, join, 0)) != hipSuccess)
            return fail(ABM_EDEVICE, "stream join");
    }
    if (pl->timing && !tev.empty()) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "timing sync");
        for (auto& te : tev) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, pl->events[te.second], pl->events[te.second + 1]);
            if (e != hipSuccess) return hip_fail(e, "event time");
            (te.first == 0 ? S.far_ms : S.chain_ms) += ms;
        }
    }
    if (stats) *stats = S;
    return ABM_OK;
}

extern "C" abm_status abm_plan_timing(abm_plan_t* pl, int32_t enable)
{
    if (!pl) return fail(ABM_EINVAL, "plan is NULL");
    pl->timing = enable != 0;
    return ABM_OK;
}
