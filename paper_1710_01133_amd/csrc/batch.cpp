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
        if (g.traj_host) (void)hipHostFree(g.traj_host);
        if (g.traj_ev) (void)hipEventDestroy(g.traj_ev);
    }
    pl->groups.clear();
    dev_free(pl->ffpart);
    pl->ffpart = nullptr;
}

abm_status batch_setup(abm_plan_s* pl)
{
    hipStream_t st = pl->ctx->stream;
    int L = env_int("ABM_BLOCK_L", 256);
    if (!valid_L(L)) return fail(ABM_EINVAL, "ABM_BLOCK_L=%d not in {64,128,256,512}", L);
    int kchunk = env_int("ABM_KCHUNK", 2048);
    if (kchunk < 64 || kchunk % 64) return fail(ABM_EINVAL, "ABM_KCHUNK=%d must be a multiple of 64", kchunk);
    while (kchunk > 64 && far_lds_bytes(L, kchunk, ABM_FAR_FP64) > 65536) kchunk /= 2;
    pl->L = L;
    pl->kchunk = kchunk;

    // groups: (weight table, rhs, precision); members sorted by N descending
    std::map<std::tuple<int, int, int>, int> key_to_group;
    for (int i = 0; i < pl->B; ++i) {
        const abm_problem& p = pl->shape[i];
        if (p.far_prec != ABM_FAR_FP64)
            return fail(ABM_EINVAL, "problem %d: far_prec %d is not available in this build", i,
                        p.far_prec);
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
    const int TN = far_tile_cols(L, ABM_FAR_FP64);
    size_t ff_need = 0;
    for (auto& g : pl->groups) {
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
        const int64_t kfar_max = (nblocks - 1) * L;
        const int64_t nch = (kfar_max + kchunk - 1) / kchunk;
        ff_need = std::max(ff_need, (size_t)nch * g.ldF * 2 * L * sizeof(double));
        abm_status s;
        if ((s = dev_alloc((void**)&g.F, (size_t)g.rows * g.ldF * sizeof(double), "history")))
            return s;
        hipError_t e = hipMemsetAsync(g.F, 0, (size_t)g.rows * g.ldF * sizeof(double), st);
        if (e != hipSuccess) return hip_fail(e, "history clear");
        if ((s = dev_alloc((void**)&g.traj_dev, g.members.size() * sizeof(TrajDesc), "descriptors")))
            return s;
        e = hipHostMalloc((void**)&g.traj_host, g.members.size() * sizeof(TrajDesc), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "pinned descriptors");
        e = hipEventCreateWithFlags(&g.traj_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "event");
    }
    pl->ffpart_bytes = ff_need;
    if (ff_need) {
        abm_status s = dev_alloc((void**)&pl->ffpart, ff_need, "far partials");
        if (s) return s;
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
    auto timed = [&](int kind, auto&& launch) -> hipError_t {
        if (!pl->timing) return launch();
        hipEvent_t a = ev_next(), b = ev_next();
        if (!a || !b) return hipErrorOutOfMemory;
        const int ia = (int)ev_used - 2;
        hipError_t e1 = hipEventRecord(a, st);
        if (e1 != hipSuccess) return e1;
        e1 = launch();
        if (e1 != hipSuccess) return e1;
        e1 = hipEventRecord(b, st);
        tev.push_back({kind, ia});
        return e1;
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
        Fa.F = g.F;
        Fa.ldF = g.ldF;
        Fa.kchunk = pl->kchunk;
        Fa.part = pl->ffpart;
        const int64_t nblocks = (int64_t)g.active_traj.size();
        for (int64_t m = 0; m < nblocks; ++m) {
            const int64_t kfar = m * L;
            Fa.mL = m * L;
            Fa.kfar = kfar;
            Fa.ldP = g.active_cols[m];
            if (kfar >= 1) {
                e = timed(0, [&]() { return launch_far(Fa, L, g.prec, st); });
                if (e != hipSuccess) return hip_fail(e, "far-field launch");
                ++S.far_launches;
                for (int32_t j = 0; j < g.active_traj[m]; ++j) {
                    const abm_problem& p = probs[g.members[j]];
                    const int64_t rows = std::min<int64_t>(L, p.N - m * L);
                    S.far_macs += (int64_t)p.d * rows * kfar;
                }
            }
            C.ntraj = g.active_traj[m];
            C.nchunks = (int32_t)((kfar + pl->kchunk - 1) / pl->kchunk);
            C.ldP = g.active_cols[m];
            C.mL = m * L;
            e = timed(1, [&]() { return launch_chain(C, g.rhs, L, st); });
            if (e != hipSuccess) return hip_fail(e, "chain launch");
            ++S.chain_launches;
        }
    }
    if (pl->timing && !tev.empty()) {
        e = hipEventSynchronize(pl->events[ev_used - 1]);
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
