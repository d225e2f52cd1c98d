// Autotuning of the batched method's blocking by measurement: each candidate
// plan runs one warm-up and one timed abm_solve_batch on the context's
// stream, on the caller's own problems (with scratch outputs).
#include <hip/hip_runtime.h>

#include <chrono>
#include <vector>

#include "abm.h"
#include "abm_runtime.h"

namespace abm {

namespace {

double wall_s()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Tuner {
    abm_ctx* ctx;
    const abm_problem* probs;
    int32_t B;
    std::vector<double*> outs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<abm_tune_trial> trials;
    std::vector<int32_t> narrow;            // narrow groups seen by each trial

    // one trial; returns its status (recorded with the time)
    abm_status run(const abm_tuning& cfg)
    {
        abm_tune_trial tr{};
        tr.cfg = cfg;
        tr.ms = -1.0;
        int32_t tr_narrow = 0;
        abm_plan_t* pl = nullptr;
        abm_status s = abm_plan_tuned(ctx, probs, B, &cfg, &pl);
        if (s == ABM_OK) {
            (void)abm_plan_config(pl, &tr.cfg);   // the blocking actually used
            for (const abm_tune_trial& t : trials)
                if (t.status == ABM_OK && t.cfg.block_L == tr.cfg.block_L &&
                    t.cfg.kchunk == tr.cfg.kchunk && t.cfg.max_split == tr.cfg.max_split &&
                    t.cfg.column_tiles_only == tr.cfg.column_tiles_only) {
                    abm_plan_destroy(pl);             // already measured
                    return ABM_OK;
                }
            s = abm_solve_batch(pl, probs, B, outs.data(), nullptr);
            hipError_t e = hipSuccess;
            if (s == ABM_OK && (e = hipEventRecord(ev0, ctx->stream)) != hipSuccess) s = hip_fail(e, "event");
            abm_stats st{};
            if (s == ABM_OK) s = abm_solve_batch(pl, probs, B, outs.data(), &st);
            tr_narrow = st.narrow_groups;
            if (s == ABM_OK && (e = hipEventRecord(ev1, ctx->stream)) != hipSuccess) s = hip_fail(e, "event");
            if (s == ABM_OK) s = abm_plan_check(pl);
            float ms = 0.f;
            if (s == ABM_OK && (e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) s = hip_fail(e, "event");
            if (s == ABM_OK) tr.ms = ms;
            abm_plan_destroy(pl);
        }
        tr.status = s;
        trials.push_back(tr);
        narrow.push_back(tr_narrow);
        return s;
    }

    // The fastest trial, in trial order, where a later trial replaces the
    // incumbent only when it is faster by more than kMargin: repeated solves
    // of one blocking differ by about 1%, and a choice made on noise would
    // change from run to run.
    const abm_tune_trial* best() const
    {
        constexpr double kMargin = 0.02;
        const abm_tune_trial* b = nullptr;
        for (const abm_tune_trial& t : trials)
            if (t.status == ABM_OK && (!b || t.ms < b->ms * (1.0 - kMargin))) b = &t;
        return b;
    }
};

}  // namespace

}  // namespace abm

using namespace abm;

extern "C" abm_status abm_autotune(abm_ctx* ctx, const abm_problem* probs, int32_t B, double budget_s,
                                   abm_tuning* best, abm_tune_trial* trials, int32_t max_trials,
                                   int32_t* n_trials)
{
    if (!ctx || !probs || !best) return fail(ABM_EINVAL, "NULL argument");
    if (B < 1) return fail(ABM_EINVAL, "B=%d must be >= 1", B);
    if (!(budget_s >= 0.0)) return fail(ABM_EINVAL, "budget must be >= 0 seconds");
    bool all_fp64 = true;
    for (int i = 0; i < B; ++i) {
        abm_status s = validate(probs[i], i);
        if (s) return s;
        if (probs[i].far_prec == ABM_FAR_DD)
            return fail(ABM_EINVAL, "problem %d: double-double runs on abm_solve, nothing to tune", i);
        all_fp64 &= probs[i].far_prec == ABM_FAR_FP64;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

    Tuner T;
    T.ctx = ctx;
    T.probs = probs;
    T.B = B;
    // scratch outputs, one allocation for all problems
    std::vector<int64_t> off(B);
    int64_t total = 0;
    for (int i = 0; i < B; ++i) {
        off[i] = total;
        total += n_out(probs[i].N, probs[i].out_stride) * probs[i].d;
    }
    double* scratch = nullptr;
    abm_status s = dev_alloc((void**)&scratch, (size_t)total * sizeof(double), "tuning outputs");
    if (s) return s;
    for (int i = 0; i < B; ++i) T.outs.push_back(scratch + off[i]);
    if ((e = hipEventCreate(&T.ev0)) != hipSuccess || (e = hipEventCreate(&T.ev1)) != hipSuccess) {
        if (T.ev0) (void)hipEventDestroy(T.ev0);
        dev_free(scratch);
        return hip_fail(e, "event");
    }

    const double t0 = wall_s();
    auto in_budget = [&]() { return wall_s() - t0 < budget_s; };
    // stage 1: block length (always at least one trial)
    std::vector<int> Ls = {256, 128, 512};
    if (all_fp64) Ls.push_back(64);
    for (size_t i = 0; i < Ls.size(); ++i) {
        if (i > 0 && !in_budget()) break;
        abm_tuning c{};
        c.block_L = Ls[i];
        (void)T.run(c);
    }
    // stage 2: split count (fewest partial slices first: a larger count has to
    // win by the margin), stage 3: chunk, at the best so far
    const int splits[] = {2, 4, 16};
    for (int sp : splits) {
        const abm_tune_trial* b = T.best();
        if (!b || !in_budget()) break;
        abm_tuning c = b->cfg;
        c.max_split = sp;
        (void)T.run(c);
    }
    const int chunks[] = {1024, 4096, 8192};
    for (int kc : chunks) {
        const abm_tune_trial* b = T.best();
        if (!b || !in_budget()) break;
        abm_tuning c = b->cfg;
        c.kchunk = kc;
        (void)T.run(c);
    }
    // stage 4: column tiles for every group instead of the blocked convolution
    if (const abm_tune_trial* b = T.best()) {
        if (in_budget() && T.narrow[b - T.trials.data()] > 0) {
            abm_tuning c = b->cfg;
            c.column_tiles_only = 1;
            (void)T.run(c);
        }
    }
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipEventDestroy(T.ev0);
    (void)hipEventDestroy(T.ev1);
    dev_free(scratch);

    const int32_t n = (int32_t)T.trials.size();
    if (n_trials) *n_trials = n;
    if (trials)
        for (int32_t i = 0; i < n && i < max_trials; ++i) trials[i] = T.trials[i];
    const abm_tune_trial* b = T.best();
    if (!b) return fail(ABM_EDEVICE, "no blocking could be run for these problems");
    *best = b->cfg;
    return ABM_OK;
}
