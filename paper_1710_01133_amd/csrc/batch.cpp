// Blocked batch path: plan-time grouping, sizing and tick schedule, and the
// launch sequence of abm_solve_batch.
//
// Trajectories are grouped by (weight table of each component = the orders,
// right-hand side, far precision).  All groups advance in lockstep ticks: at
// tick t every group still running steps its block m = t (chain) while the
// far field of its block t+1 is computed on a second stream.  One far launch
// per precision class and one chain launch cover all groups of a tick,
// whatever their alpha, N or parameters (work items in device memory).
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

int group_split_plan(const Group& g, int64_t kfar, int L, int kchunk, int max_split, int* nchunks,
                     int* chunks_per_split);

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

void free_group(Group& g)
{
    dev_free(g.F);
    dev_free(g.F32);
    for (int i = 0; i < 3; ++i) dev_free(g.Fh[i]);
    dev_free(g.Fsc);
    for (int i = 0; i < 3; ++i) dev_free(g.Fq[i]);
    dev_free(g.Fqs);
    dev_free(g.traj_dev);
    dev_free(g.accn);
    dev_free(g.part[0]);
    if (g.traj_host) (void)hipHostFree(g.traj_host);
    if (g.traj_ev) (void)hipEventDestroy(g.traj_ev);
    g = Group{};
}

void batch_teardown(abm_plan_s* pl)
{
    if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->graph_exec = nullptr;
    pl->graph = nullptr;
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    pl->cap_stream = nullptr;
    for (hipEvent_t ev : pl->events) (void)hipEventDestroy(ev);
    pl->events.clear();
    for (auto& g : pl->groups) free_group(g);
    pl->groups.clear();
    dev_free(pl->groups_dev);
    dev_free(pl->far_items_dev);
    dev_free(pl->chain_items_dev);
    dev_free(pl->init_items_dev);
    pl->groups_dev = nullptr;
    pl->far_items_dev = nullptr;
    pl->chain_items_dev = nullptr;
    pl->init_items_dev = nullptr;
    for (hipEvent_t ev : pl->sync_events) (void)hipEventDestroy(ev);
    pl->sync_events.clear();
    if (pl->far_stream) (void)hipStreamDestroy(pl->far_stream);
    pl->far_stream = nullptr;

}

// Reduced copies of a weight table for far precision prec (once per table).
abm_status ensure_reduced_weights(WeightTable& W, int prec, hipStream_t st)
{
    abm_status s;
    hipError_t e;
    const int64_t wn = W.n + kWeightPad;
    if ((prec == ABM_FAR_FP32 || prec == ABM_FAR_FP16X3) && !W.b32) {
        if ((s = dev_alloc((void**)&W.b32, wn * sizeof(float), "float weights")) ||
            (s = dev_alloc((void**)&W.a32, wn * sizeof(float), "float weights")))
            return s;
        uint16_t* none[3] = {nullptr, nullptr, nullptr};
        if ((e = launch_weights_lowp(wn, W.b, W.a, W.b32, W.a32, none, none, st)) != hipSuccess)
            return hip_fail(e, "weight conversion");
    }
    if ((prec == ABM_FAR_BF16X3 || prec == ABM_FAR_BF16X6) && !W.bh[0]) {
        for (int tt = 0; tt < 3; ++tt)
            if ((s = dev_alloc((void**)&W.bh[tt], wn * sizeof(uint16_t), "bf16 weights")) ||
                (s = dev_alloc((void**)&W.ah[tt], wn * sizeof(uint16_t), "bf16 weights")))
                return s;
        if ((e = launch_weights_lowp(wn, W.b, W.a, nullptr, nullptr, W.bh, W.ah, st)) != hipSuccess)
            return hip_fail(e, "weight conversion");
    }
    return ABM_OK;
}

// Device memory of one group: history (+ reduced copy), carried sums, far
// partial double buffer, descriptors.  nsplit_max bounds the partial slices.
abm_status alloc_group(Group& g, int L, int nsplit_max, hipStream_t st)
{
    abm_status s;
    hipError_t e;
    const size_t nm = g.members.size();
    if ((s = dev_alloc((void**)&g.F, (size_t)g.rows * g.ldF * sizeof(double), "history")))
        return s;
    if ((e = hipMemsetAsync(g.F, 0, (size_t)g.rows * g.ldF * sizeof(double), st)) != hipSuccess)
        return hip_fail(e, "history clear");
    if (g.prec == ABM_FAR_FP32) {
        const size_t bytes = (size_t)g.rows * g.ldF * sizeof(float);
        if ((s = dev_alloc((void**)&g.F32, bytes, "float history"))) return s;
        if ((e = hipMemsetAsync(g.F32, 0, bytes, st)) != hipSuccess) return hip_fail(e, "clear");
    } else if (g.prec == ABM_FAR_BF16X3 || g.prec == ABM_FAR_BF16X6 || g.prec == ABM_FAR_FP16X3) {
        const int terms = g.prec == ABM_FAR_BF16X6 ? 3 : 2;
        const size_t bytes = (size_t)((g.rows + 7) / 8) * g.ldF * 8 * sizeof(uint16_t);
        for (int tt = 0; tt < terms; ++tt) {
            if ((s = dev_alloc((void**)&g.Fh[tt], bytes, "split history"))) return s;
            if ((e = hipMemsetAsync(g.Fh[tt], 0, bytes, st)) != hipSuccess) return hip_fail(e, "clear");
        }
        if (g.prec == ABM_FAR_FP16X3) {
            const size_t sb = (size_t)(g.rows / 32 + 1) * g.ldF * sizeof(float);
            if ((s = dev_alloc((void**)&g.Fsc, sb, "history scales"))) return s;
            if ((e = hipMemsetAsync(g.Fsc, 0, sb, st)) != hipSuccess) return hip_fail(e, "clear");
        }
    } else if (g.prec == ABM_FAR_I8) {
        const size_t bytes = (size_t)((g.rows + 15) / 16) * g.ldF * 16;
        for (int i = 0; i < 3; ++i) {
            if ((s = dev_alloc((void**)&g.Fq[i], bytes, "int8 history"))) return s;
            if ((e = hipMemsetAsync(g.Fq[i], 0, bytes, st)) != hipSuccess) return hip_fail(e, "clear");
        }
        const size_t sb = (size_t)(g.rows / L + 1) * g.ldF * sizeof(double);
        if ((s = dev_alloc((void**)&g.Fqs, sb, "history scales"))) return s;
        if ((e = hipMemsetAsync(g.Fqs, 0, sb, st)) != hipSuccess) return hip_fail(e, "clear");
    }
    if ((s = dev_alloc((void**)&g.traj_dev, nm * sizeof(TrajDesc), "descriptors"))) return s;
    if ((s = dev_alloc((void**)&g.accn, nm * 2 * g.d * L * sizeof(double), "carried sums"))) return s;
    g.nsplit_cap = std::max(nsplit_max, 1);
    g.part_half = (size_t)g.nsplit_cap * g.ldF * 2 * L;
    if ((s = dev_alloc((void**)&g.part[0], 2 * g.part_half * sizeof(double), "far partials"))) return s;
    g.part[1] = g.part[0] + g.part_half;
    if ((e = hipHostMalloc((void**)&g.traj_host, nm * sizeof(TrajDesc), hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "pinned descriptors");
    if ((e = hipEventCreateWithFlags(&g.traj_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "event");
    return ABM_OK;
}

GroupDev group_dev(const Group& g, const WeightTable* const W[4])
{
    GroupDev d{};
    for (int c = 0; c < 4; ++c) {
        CompWeights& w = d.w[c];
        w.b = W[c]->b;
        w.a = W[c]->a;
        w.c = W[c]->c;
        w.gam = W[c]->gam;
        w.b32 = W[c]->b32;
        w.a32 = W[c]->a32;
        for (int i = 0; i < 3; ++i) {
            w.bh[i] = W[c]->bh[i];
            w.ah[i] = W[c]->ah[i];
        }
        w.alpha = W[c]->alpha;
    }
    for (int i = 0; i < 3; ++i) d.Fh[i] = g.Fh[i];
    d.Fsc = g.Fsc;
    for (int i = 0; i < 3; ++i) d.Fq[i] = g.Fq[i];
    d.Fqs = g.Fqs;
    d.F = g.F;
    d.F32 = g.F32;
    d.ldF = g.ldF;
    d.rows = g.rows;
    d.accn = g.accn;
    d.part[0] = g.part[0];
    d.part[1] = g.part[1];
    d.traj = g.traj_dev;
    d.d = g.d;
    d.narrow = g.narrow ? 1 : 0;
    d.per_comp = g.per_comp ? 1 : 0;
    d.deriv = g.deriv;
    d.status = g.status;
    return d;
}

void group_layout(Group& g, int L)
{
    const int64_t nm = (int64_t)g.members.size();
    const int TN = far_tile_cols(L, g.prec);
    g.cols = nm * g.d;
    g.col0.resize(nm);
    if (g.per_comp) {
        // component-major: each component's columns form a block that starts
        // on a tile (and 16-column) boundary unless the group is narrow
        g.ldC = g.narrow ? nm : round_up(nm, std::max(TN, 16));
        g.ldF = g.ldC * g.d;
        for (int64_t j = 0; j < nm; ++j) g.col0[j] = (int32_t)j;
    } else {
        g.ldC = 1;
        g.ldF = g.narrow ? g.cols : round_up(g.cols, TN);
        for (int64_t j = 0; j < nm; ++j) g.col0[j] = (int32_t)(j * g.d);
    }
}

// Work items of group g (index gi) when it is at block m: the far field of
// block m+1 and the chains of block m.  memberN holds the members' N in the
// group's (descending) order, so the members still running form a prefix.
void block_items(const Group& g, int gi, int64_t m, int L, int kchunk, int max_split,
                 const std::vector<int64_t>& memberN, std::vector<FarItem>* far,
                 std::vector<ChainItem>* chain)
{
    const int TN = far_tile_cols(L, g.prec);
    const int64_t nblocks = (g.nmax + L - 1) / L;
    auto active = [&](int64_t mm) {
        int32_t cnt = 0;
        for (int64_t N : memberN)
            if (N > mm * L) ++cnt;
        return cnt;
    };
    const int64_t mf = m + 1;
    if (far && mf < nblocks && mf >= 2) {
        FarItem it{};
        it.group = gi;
        it.kfar = (mf - 1) * L;
        it.mL = mf * L;
        it.nsplit = group_split_plan(g, it.kfar, L, kchunk, max_split, &it.nchunks,
                                     &it.chunks_per_split);
        const int64_t na = active(mf);
        if (g.per_comp) {
            // one item per component: its column block, its weight tables;
            // the partial slices keep the group's full column stride
            it.ldP = g.ldF;
            it.ncols = (int32_t)na;
            it.ncoltiles = g.narrow ? hankel_tiles(na, L) : (int32_t)((na + TN - 1) / TN);
            for (int c = 0; c < g.d; ++c) {
                it.comp = c;
                it.coff = (int32_t)(c * g.ldC);
                far->push_back(it);
            }
        } else {
            if (g.narrow) {
                it.ldP = na * g.d;
                it.ncoltiles = hankel_tiles(it.ldP, L);
            } else {
                it.ldP = round_up(na * g.d, TN);
                it.ncoltiles = (int32_t)(it.ldP / TN);
            }
            it.ncols = (int32_t)(na * g.d);
            far->push_back(it);
        }
    }
    if (chain && m < nblocks) {
        int nsp = 0, nc = 0, cps = 0;
        if (m >= 2) nsp = group_split_plan(g, (m - 1) * L, L, kchunk, max_split, &nc, &cps);
        const int32_t na = active(m);
        const int64_t ldP = g.per_comp ? g.ldF
                          : g.narrow  ? (int64_t)na * g.d
                                      : round_up((int64_t)na * g.d, TN);
        for (int32_t j = 0; j < na; ++j) {
            ChainItem c{};
            c.group = gi;
            c.member = j;
            c.kind = chain_kind(g.rhs, g.per_comp);
            c.nsplit = nsp;
            c.mL = m * L;
            c.ldP = ldP;
            chain->push_back(c);
        }
    }
}

int group_split_plan(const Group& g, int64_t kfar, int L, int kchunk, int max_split, int* nchunks,
                     int* chunks_per_split)
{
    if (g.narrow)
        return hankel_split_plan(kfar, L, g.split_cap > 0 ? g.split_cap : max_split, nchunks,
                                 chunks_per_split);
    return far_split_plan(kfar, kchunk, max_split, nchunks, chunks_per_split);
}

int64_t group_far_split_max(const Group& g, int L, int kchunk, int max_split)
{
    const int64_t nblocks = (g.nmax + L - 1) / L;
    const int64_t kfar_max = nblocks >= 2 ? (nblocks - 2) * L : 0;   // far(m) covers (m-1)L
    if (g.narrow) return hankel_split_bound(kfar_max, L, g.split_cap > 0 ? g.split_cap : max_split);
    return far_split_bound(kfar_max, kchunk, max_split);
}

abm_status choose_blocking(abm_plan_s* pl, const abm_problem* probs, int B)
{
    const abm_tuning& T = pl->tune;
    int L = T.block_L ? T.block_L : env_int("ABM_BLOCK_L", 256);
    if (!valid_L(L)) return fail(ABM_EINVAL, "block length %d not in {64,128,256,512}", L);
    for (int i = 0; i < B; ++i) {
        if (probs[i].far_prec != ABM_FAR_FP64 && L < 128)
            return fail(ABM_EINVAL, "problem %d: reduced-precision far field needs block length >= 128", i);
        if (probs[i].far_prec == ABM_FAR_I8 && L > 256)
            return fail(ABM_EINVAL, "problem %d: the int8 far field needs block length 128 or 256", i);
    }
    int kchunk = T.kchunk ? T.kchunk : env_int("ABM_KCHUNK", 2048);
    if (kchunk < 512 || kchunk % 512 || kchunk > (1 << 20))
        return fail(ABM_EINVAL, "history chunk %d must be a multiple of 512 (at most 2^20)", kchunk);
    // largest chunk whose LDS footprint fits every precision used
    for (int prec : kBlockedPrecs)
        while (kchunk > 512 && far_lds_bytes(L, kchunk, prec) > kMaxLds) kchunk -= 512;
    pl->L = L;
    pl->kchunk = kchunk;
    pl->max_split = T.max_split ? T.max_split : env_int("ABM_MAX_SPLIT", 8);
    if (pl->max_split < 1 || pl->max_split > 4096)
        return fail(ABM_EINVAL, "split count %d out of range 1..4096", pl->max_split);
    pl->allow_narrow = !T.column_tiles_only && env_int("ABM_NARROW", 1) != 0;
    return ABM_OK;
}

abm_status batch_setup(abm_plan_s* pl)
{
    hipStream_t st = pl->ctx->stream;
    abm_status s = choose_blocking(pl, pl->shape.data(), pl->B);
    if (s) return s;
    const int L = pl->L, kchunk = pl->kchunk;

    // groups: (weight table of each component, rhs, precision); members
    // sorted by N descending
    std::map<std::tuple<int, int, int, int, int, int>, int> key_to_group;
    for (int i = 0; i < pl->B; ++i) {
        const abm_problem& p = pl->shape[i];
        const int* tb = &pl->table_of[(size_t)i * 4];
        auto key = std::make_tuple(tb[0], tb[1], tb[2], tb[3], p.rhs, p.far_prec);
        auto it = key_to_group.find(key);
        if (it == key_to_group.end()) {
            Group g{};
            for (int c = 0; c < 4; ++c) g.table[c] = tb[c];
            g.per_comp = orders_differ(p);
            g.deriv = deriv_mask(p);
            g.rhs = p.rhs;
            g.d = p.d;
            g.prec = p.far_prec;
            pl->groups.push_back(g);
            it = key_to_group.emplace(key, (int)pl->groups.size() - 1).first;
        }
        pl->groups[it->second].members.push_back(i);
    }
    std::vector<GroupDev> gdev;
    int64_t ticks = 0;
    int n_narrow = 0;
    for (auto& g : pl->groups) {
        g.cols = (int64_t)g.members.size() * g.d;
        g.narrow = pl->allow_narrow && hankel_fits(g.prec, g.cols, L);
        n_narrow += g.narrow ? 1 : 0;
    }
    // A narrow group's convolution is a few tiles wide, so its history is
    // split over more workgroups: about 1024 in total over the narrow groups
    // (a single long trajectory gets 256), never fewer than the plan's count.
    const int narrow_split =
        n_narrow ? std::max(pl->max_split, std::min(256, 1024 / n_narrow)) : pl->max_split;
    for (auto& g : pl->groups) {
        std::stable_sort(g.members.begin(), g.members.end(),
                         [&](int x, int y) { return pl->shape[x].N > pl->shape[y].N; });
        g.nmax = pl->shape[g.members[0]].N;
        if (g.narrow) g.split_cap = narrow_split;
        group_layout(g, L);
        g.rows = g.nmax + 1 + L;
        ticks = std::max(ticks, (g.nmax + L - 1) / L);
        const WeightTable* W[4];
        for (int c = 0; c < 4; ++c) {
            if ((s = ensure_reduced_weights(pl->tables[g.table[c]], g.prec, st))) return s;
            W[c] = &pl->tables[g.table[c]];
        }
        if ((s = alloc_group(g, L, (int)group_far_split_max(g, L, kchunk, pl->max_split), st))) return s;
        gdev.push_back(group_dev(g, W));
    }

    // static tick schedule: far items by precision class, chain items by rhs
    const int ngroups = (int)pl->groups.size();
    std::vector<std::vector<int64_t>> memberN(ngroups);
    for (int gi = 0; gi < ngroups; ++gi)
        for (int idx : pl->groups[gi].members) memberN[gi].push_back(pl->shape[idx].N);
    pl->ticks = ticks;
    pl->far_spans.assign((size_t)ticks * kFarClasses, Span{});
    pl->chain_spans.assign((size_t)ticks * kChainKinds, Span{});
    std::vector<FarItem> far_all;
    std::vector<ChainItem> chain_all, init_all;
    for (int64_t t = 0; t < ticks; ++t) {
        for (int cls = 0; cls < kFarClasses; ++cls) {
            Span& sp = pl->far_spans[t * kFarClasses + cls];
            sp.offset = (int64_t)far_all.size();
            for (int gi = 0; gi < ngroups; ++gi)
                if (far_class(pl->groups[gi].prec, pl->groups[gi].narrow) == cls)
                    block_items(pl->groups[gi], gi, t, L, kchunk, pl->max_split, memberN[gi],
                                &far_all, nullptr);
            sp.count = (int32_t)((int64_t)far_all.size() - sp.offset);
            for (int64_t k = sp.offset; k < (int64_t)far_all.size(); ++k) {
                sp.max_x = std::max(sp.max_x, far_all[k].ncoltiles);
                sp.max_y = std::max(sp.max_y, far_all[k].nsplit);
                sp.max_cols = std::max(sp.max_cols, far_all[k].ncols);
            }
        }
        for (int kind = 0; kind < kChainKinds; ++kind) {
            Span& sp = pl->chain_spans[t * kChainKinds + kind];
            sp.offset = (int64_t)chain_all.size();
            for (int gi = 0; gi < ngroups; ++gi)
                if (chain_kind(pl->groups[gi].rhs, pl->groups[gi].per_comp) == kind) {
                    const size_t c0 = chain_all.size();
                    block_items(pl->groups[gi], gi, t, L, kchunk, pl->max_split, memberN[gi],
                                nullptr, &chain_all);
                    // a narrow group's slices are summed into the first one
                    // after its far field (launch_far_reduce)
                    if (pl->groups[gi].narrow)
                        for (size_t k = c0; k < chain_all.size(); ++k)
                            chain_all[k].nsplit = std::min(chain_all[k].nsplit, 1);
                }
            sp.count = (int32_t)((int64_t)chain_all.size() - sp.offset);
        }
    }
    pl->init_spans.assign(kRhsCount, Span{});
    for (int rhs = 0; rhs < kRhsCount; ++rhs) {
        Span& sp = pl->init_spans[rhs];
        sp.offset = (int64_t)init_all.size();
        for (int gi = 0; gi < ngroups; ++gi) {
            const Group& g = pl->groups[gi];
            if (g.rhs != rhs) continue;
            for (size_t j = 0; j < g.members.size(); ++j) {
                ChainItem c{};
                c.group = gi;
                c.member = (int32_t)j;
                init_all.push_back(c);
            }
        }
        sp.count = (int32_t)((int64_t)init_all.size() - sp.offset);
    }
    // every item must fit its group's partial buffers (checked, not assumed)
    for (const FarItem& it : far_all) {
        const Group& g = pl->groups[it.group];
        if (it.nsplit > g.nsplit_cap || it.ldP > g.ldF)
            return fail(ABM_EDEVICE, "internal: far item exceeds the partial buffer of group %d", it.group);
        if (g.narrow && !hankel_fits(g.prec, it.ncols, L))
            return fail(ABM_EDEVICE, "internal: narrow far item of group %d has too many columns", it.group);
        if (it.coff + (int64_t)it.ncols > g.ldF || (!g.narrow && it.coff % 16))
            return fail(ABM_EDEVICE, "internal: far item of group %d outside its columns", it.group);
    }
    for (const ChainItem& it : chain_all)
        if (it.nsplit > pl->groups[it.group].nsplit_cap)
            return fail(ABM_EDEVICE, "internal: chain item exceeds the partial buffer of group %d", it.group);
    hipError_t e;
    if ((s = dev_alloc((void**)&pl->groups_dev, gdev.size() * sizeof(GroupDev), "group table")) ||
        (s = dev_alloc((void**)&pl->far_items_dev, std::max<size_t>(1, far_all.size()) * sizeof(FarItem), "far items")) ||
        (s = dev_alloc((void**)&pl->chain_items_dev, std::max<size_t>(1, chain_all.size()) * sizeof(ChainItem), "chain items")) ||
        (s = dev_alloc((void**)&pl->init_items_dev, std::max<size_t>(1, init_all.size()) * sizeof(ChainItem), "init items")))
        return s;
    if ((e = hipMemcpy(pl->groups_dev, gdev.data(), gdev.size() * sizeof(GroupDev), hipMemcpyHostToDevice)) ||
        (!far_all.empty() && (e = hipMemcpy(pl->far_items_dev, far_all.data(), far_all.size() * sizeof(FarItem), hipMemcpyHostToDevice))) ||
        (e = hipMemcpy(pl->chain_items_dev, chain_all.data(), chain_all.size() * sizeof(ChainItem), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(pl->init_items_dev, init_all.data(), init_all.size() * sizeof(ChainItem), hipMemcpyHostToDevice)))
        return hip_fail(e, "schedule upload");
    // useful far-field MACs of the schedule (reported in abm_stats), per tick
    pl->far_macs = 0;
    std::vector<int64_t> tick_macs(ticks, 0);
    for (int64_t t = 0; t < ticks; ++t)
        for (int cls = 0; cls < kFarClasses; ++cls) {
            const Span& sp = pl->far_spans[t * kFarClasses + cls];
            for (int64_t k = sp.offset; k < sp.offset + sp.count; ++k) {
                const FarItem& it = far_all[k];
                const Group& g = pl->groups[it.group];
                for (int64_t N : memberN[it.group]) {
                    if (N <= it.mL) continue;
                    tick_macs[t] += (int64_t)(g.per_comp ? 1 : g.d) * std::min<int64_t>(L, N - it.mL) * it.kfar;
                }
            }
        }
    int64_t max_tick = 0;
    for (int64_t t = 0; t < ticks; ++t) {
        pl->far_macs += tick_macs[t];
        max_tick = std::max(max_tick, tick_macs[t]);
    }
    // Chains are spread one wave per SIMD in the ticks whose far field (the
    // launch running beside them) is below this share (percent) of the
    // largest one, and packed two waves per SIMD in the others.  With the far
    // fields of consecutive ticks overlapping (the streams alternate), a chain
    // wave beside one far-field wave on every SIMD measured best in every
    // tick, so by default (101) every tick spreads.
    const int spread_pct = env_int("ABM_CHAIN_SPREAD", 101);
    pl->chain_spread.assign(ticks, 0);
    for (int64_t t = 0; t < ticks; ++t)
        pl->chain_spread[t] = (int64_t)100 * tick_macs[t] < (int64_t)spread_pct * max_tick ? 1 : 0;
    pl->overlap = env_int("ABM_OVERLAP", 1) != 0;
    if (pl->overlap) {
        e = hipStreamCreateWithFlags(&pl->far_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "far stream");
    }
    return ABM_OK;
}

namespace {

// Enqueues the launch sequence of one blocked solve after its descriptor
// upload: the chain initialisation, then per tick the far field of the next
// block on the far stream and the chains of this block on the given stream,
// ordered by events so that far(t+1) overlaps chain(t).  Runs eagerly
// (optionally bracketing every launch with timing events) or under capture.
struct TickEnqueuer {
    abm_plan_s* pl;
    bool timing;
    std::vector<std::pair<int, int>> tev;   // (0 far | 1 chain, index of the start event)
    size_t ev_used = 0, sync_used = 0;
    int64_t far_launches = 0, chain_launches = 0;

    TickEnqueuer(abm_plan_s* p, bool t) : pl(p), timing(t) {}

    hipEvent_t timing_event()
    {
        if (ev_used == pl->events.size()) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return nullptr;
            pl->events.push_back(ev);
        }
        return pl->events[ev_used++];
    }
    // ordering events (no timing), reused across calls
    hipEvent_t sync_event()
    {
        if (sync_used == pl->sync_events.size()) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
            pl->sync_events.push_back(ev);
        }
        return pl->sync_events[sync_used++];
    }
    template <class Launch>
    hipError_t timed(int kind, hipStream_t sx, Launch&& launch)
    {
        if (!timing) return launch();
        hipEvent_t a = timing_event(), b = timing_event();
        if (!a || !b) return hipErrorOutOfMemory;
        const int ia = (int)ev_used - 2;
        hipError_t e = hipEventRecord(a, sx);
        if (e != hipSuccess) return e;
        if ((e = launch()) != hipSuccess) return e;
        e = hipEventRecord(b, sx);
        tev.push_back({kind, ia});
        return e;
    }

    abm_status run(hipStream_t st)
    {
        hipError_t e;
        const int L = pl->L;
        for (int rhs = 0; rhs < kRhsCount; ++rhs) {
            const Span& sp = pl->init_spans[rhs];
            if (!sp.count) continue;
            e = launch_chain_init(pl->groups_dev, pl->init_items_dev + sp.offset, sp.count, rhs, st);
            if (e != hipSuccess) return hip_fail(e, "chain init launch");
        }
        hipStream_t s1 = pl->overlap ? pl->far_stream : st;
        hipEvent_t fork = sync_event();
        if (!fork) return fail(ABM_EDEVICE, "event pool");
        if ((e = hipEventRecord(fork, st)) != hipSuccess || (e = hipStreamWaitEvent(s1, fork, 0)) != hipSuccess)
            return hip_fail(e, "stream fork");
        // The two streams swap roles every tick: tick t runs chain(t) on S[t mod 2]
        // and the far field of block t+1 on the other stream, i.e. after chain(t-1)
        // (its input) in stream order; chain(t) follows the far field of its block
        // in stream order and waits for chain(t-1) by event.  Each tick thus has
        // one cross-stream wait.  The partial slices alternate by block parity, so
        // far(t+1) overwrites the slices of block t-1 only after chain(t-1), the
        // stream's previous work, has read them.
        const bool alt = pl->overlap && env_int("ABM_ALT_STREAMS", 1) != 0;
        hipEvent_t ev_chain_prev = nullptr, ev_far_prev = nullptr;
        for (int64_t t = 0; t < pl->ticks; ++t) {
            hipStream_t sc = st, sf = s1;
            if (alt && (t & 1)) std::swap(sc, sf);
            bool any_far = false;
            for (int cls = 0; cls < kFarClasses; ++cls)
                if (pl->far_spans[t * kFarClasses + cls].count) any_far = true;
            hipEvent_t ev_far = nullptr;
            if (any_far) {
                if (!alt && ev_chain_prev && (e = hipStreamWaitEvent(sf, ev_chain_prev, 0)) != hipSuccess)
                    return hip_fail(e, "stream wait");
                for (int cls = 0; cls < kFarClasses; ++cls) {
                    const Span& sp = pl->far_spans[t * kFarClasses + cls];
                    if (!sp.count) continue;
                    e = timed(0, sf, [&]() {
                        return launch_far(pl->groups_dev, pl->far_items_dev + sp.offset, sp.count,
                                          sp.max_x, sp.max_y, pl->kchunk, L, cls, sf);
                    });
                    if (e != hipSuccess) return hip_fail(e, "far-field launch");
                    ++far_launches;
                    if (is_narrow_class(cls) && sp.max_y > 1 &&
                        (e = launch_far_reduce(pl->groups_dev, pl->far_items_dev + sp.offset, sp.count,
                                               sp.max_cols, L, sf)) != hipSuccess)
                        return hip_fail(e, "partial reduction launch");
                }
                if (!alt) {
                    ev_far = sync_event();
                    if (!ev_far || (e = hipEventRecord(ev_far, sf)) != hipSuccess)
                        return fail(ABM_EDEVICE, "far event");
                }
            }
            if (alt) {
                if (ev_chain_prev && (e = hipStreamWaitEvent(sc, ev_chain_prev, 0)) != hipSuccess)
                    return hip_fail(e, "stream wait");
            } else if (ev_far_prev && (e = hipStreamWaitEvent(sc, ev_far_prev, 0)) != hipSuccess) {
                return hip_fail(e, "stream wait");
            }
            // chains of every kind: one launch (one kernel switching per wave
            // when the tick mixes systems), so they run side by side
            int nkind = 0, nch = 0, nw = 1;
            int64_t off0 = -1;
            for (int kind = 0; kind < kChainKinds; ++kind) {
                const Span& sp = pl->chain_spans[t * kChainKinds + kind];
                if (!sp.count) continue;
                ++nkind;
                if (off0 < 0) off0 = sp.offset;
                nch += sp.count;
                nw = std::max(nw, chain_tables(kind));
            }
            if (nkind > 1) {
                e = timed(1, sc, [&]() {
                    return launch_chain_mixed(pl->groups_dev, pl->chain_items_dev + off0, nch, L,
                                              nw, pl->status, sc);
                });
                if (e != hipSuccess) return hip_fail(e, "chain launch");
                ++chain_launches;
            } else {
                for (int kind = 0; kind < kChainKinds; ++kind) {
                    const Span& sp = pl->chain_spans[t * kChainKinds + kind];
                    if (!sp.count) continue;
                    e = timed(1, sc, [&]() {
                        return launch_chain(pl->groups_dev, pl->chain_items_dev + sp.offset, sp.count,
                                            kind, L, pl->chain_spread[t] != 0, pl->status, sc);
                    });
                    if (e != hipSuccess) return hip_fail(e, "chain launch");
                    ++chain_launches;
                }
            }
            ev_chain_prev = sync_event();
            if (!ev_chain_prev || (e = hipEventRecord(ev_chain_prev, sc)) != hipSuccess)
                return fail(ABM_EDEVICE, "chain event");
            ev_far_prev = ev_far;
        }
        hipEvent_t join = sync_event();
        if (!join || (e = hipEventRecord(join, s1)) != hipSuccess ||
            (e = hipStreamWaitEvent(st, join, 0)) != hipSuccess)
            return fail(ABM_EDEVICE, "stream join");
        return ABM_OK;
    }
};

// Records the launch sequence once into a graph, from a private origin stream
// so that nothing of the caller's stream is captured.  Every pointer the
// kernels use is fixed by the plan (per-solve data reaches them through the
// descriptors uploaded before each launch), so the graph stays valid for the
// plan's lifetime.
abm_status capture_ticks(abm_plan_s* pl)
{
    hipError_t e;
    if (!pl->cap_stream &&
        (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "capture stream");
    if ((e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "begin capture");
    TickEnqueuer q(pl, false);
    const abm_status s = q.run(pl->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiateWithFlags(&pl->graph_exec, g, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        pl->graph_exec = nullptr;
        return hip_fail(e, "graph instantiate");
    }
    pl->graph = g;
    pl->graph_far_launches = q.far_launches;
    pl->graph_chain_launches = q.chain_launches;
    return ABM_OK;
}

}  // namespace

}  // namespace abm

using namespace abm;

extern "C" abm_status abm_solve_batch(abm_plan_t* pl, const abm_problem* probs, int32_t B,
                                      double* const* y_out, abm_stats* stats)
{
    if (!pl || !probs || !y_out) return fail(ABM_EINVAL, "NULL argument");
    if (pl->dd) return fail(ABM_EINVAL, "a double-double plan runs on abm_solve only");
    if (B != pl->B) return fail(ABM_EINVAL, "B=%d but the plan was made for %d problems", B, pl->B);
    for (int i = 0; i < B; ++i) {
        abm_status s = validate(probs[i], i);
        if (s) return s;
        const abm_problem& a = probs[i];
        const abm_problem& b = pl->shape[i];
        if (a.rhs != b.rhs || a.d != b.d || !same_orders(a, b) || a.N != b.N ||
            a.far_prec != b.far_prec || a.out_stride != b.out_stride)
            return fail(ABM_EINVAL, "problem %d does not match the plan", i);
        if (!y_out[i]) return fail(ABM_EINVAL, "y_out[%d] is NULL", i);
    }
    hipError_t e = hipSetDevice(pl->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = pl->ctx->stream;
    abm_stats S{};
    S.block_L = pl->L;
    S.n_groups = (int32_t)pl->groups.size();
    for (const Group& g : pl->groups) S.narrow_groups += g.narrow ? 1 : 0;
    S.far_macs = pl->far_macs;

    // per-solve descriptors (x0, p, h, outputs) through the pinned staging copies
    for (auto& g : pl->groups) {
        if (g.traj_ev_live) {
            e = hipEventSynchronize(g.traj_ev);
            if (e != hipSuccess) return hip_fail(e, "descriptor staging wait");
        }
        TrajDesc* td = g.traj_host;
        for (size_t j = 0; j < g.members.size(); ++j) {
            const abm_problem& p = probs[g.members[j]];
            TrajDesc& T = td[j];
            memset(&T, 0, sizeof T);
            for (int i = 0; i < 4; ++i) {
                T.x0[i] = p.x0[i];
                T.x1[i] = p.x1[i];
            }
            for (int i = 0; i < 8; ++i) T.p[i] = p.p[i];
            T.h = p.h;
            T.N = p.N;
            T.out_stride = p.out_stride;
            T.y_out = y_out[g.members[j]];
            T.col0 = g.col0[j];
            T.cstride = (int32_t)g.ldC;
            S.history_macs += (int64_t)p.d * p.N * (p.N + 1) / 2;
        }
        e = hipMemcpyAsync(g.traj_dev, td, g.members.size() * sizeof(TrajDesc),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        e = hipEventRecord(g.traj_ev, st);
        if (e != hipSuccess) return hip_fail(e, "descriptor event");
        g.traj_ev_live = true;
    }

    abm_status s;
    if (pl->use_graph && !pl->timing) {
        if (!pl->graph_exec && (s = capture_ticks(pl))) return s;
        e = hipGraphLaunch(pl->graph_exec, st);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        S.far_launches = pl->graph_far_launches;
        S.chain_launches = pl->graph_chain_launches;
    } else {
        TickEnqueuer q(pl, pl->timing);
        if ((s = q.run(st))) return s;
        S.far_launches = q.far_launches;
        S.chain_launches = q.chain_launches;
        if (pl->timing && !q.tev.empty()) {
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "timing sync");
            for (auto& te : q.tev) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, pl->events[te.second], pl->events[te.second + 1]);
                if (e != hipSuccess) return hip_fail(e, "event time");
                (te.first == 0 ? S.far_ms : S.chain_ms) += ms;
            }
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

extern "C" abm_status abm_plan_config(abm_plan_t* pl, abm_tuning* out)
{
    if (!pl || !out) return fail(ABM_EINVAL, "NULL argument");
    out->block_L = pl->L;
    out->kchunk = pl->kchunk;
    out->max_split = pl->max_split;
    out->column_tiles_only = pl->allow_narrow ? 0 : 1;
    return ABM_OK;
}

extern "C" abm_status abm_plan_graph(abm_plan_t* pl, int32_t enable)
{
    if (!pl) return fail(ABM_EINVAL, "plan is NULL");
    pl->use_graph = enable != 0;
    return ABM_OK;
}
