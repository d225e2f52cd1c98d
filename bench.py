"""Benchmark of the fractional ABM history sums on one MI355X.

One step = one abm_solve_batch call over the forcing sweep (B = 1024 forced
Duffing oscillators, alpha = 0.95, h = 2^-8, N = 65536, amplitudes uniform in
[0.1, 0.6] from seed 1710): weight tables resident, far-field products on the
matrix cores, near band and predictor/corrector chain, outputs every 1024th
state.  Inputs are synthetic and already in HBM when the timed region starts.

Printed: one JSON line with history MACs/s (d*N(N+1)/2 per trajectory) of the
batched path, the plain per-step path on the single 200000-step oscillator
for comparison, the far-field kernel's roofline position (live HIP-event
timing of its launches), the error against the double oracle, and the oracle
itself timed on the host cores on a bounded sample of the same sweep.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense matrix-core peaks of MI355X per operand type (int8: 5.0 POP/s)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0, "fp16x3": 2500.0,
               "i8x9": 5000.0}
EXEC_FACTOR = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "fp16x3": 3, "i8x9": 9}
DTYPE = {"fp64": "f64", "fp32": "f32 far field, f64 near/state",
         "bf16x3": "bf16x3 far field (f32 accumulate), f64 near/state",
         "bf16x6": "bf16x6 far field (f32 accumulate), f64 near/state",
         "fp16x3": "fp16x3 far field (scaled fp16 split, f32 accumulate), f64 near/state",
         "i8x9": "i8x9 far field (int8 limbs, exact i32 accumulate), f64 near/state"}


# Far-field precision of the headline: split-precision compensation on the
# int8 matrix cores (weights as four base-256 digits, the history as three,
# the nine significant digit products summed exactly in int32 and converted
# to double when a scale changes): the fastest sweep of all modes within the
# 1e-6 bar and the most accurate of the reduced ones (6.3e-8 on its worst
# member, against 4.9e-7 for the three-term bf16 split with float
# accumulation, bf16x6).  The scaled two-term fp16 split (fp16x3) carries
# about 22 significant bits of its weights: 1.1e-6 on its worst member, over
# the bar.  The other modes are reported under other_precisions.
DEFAULT_PREC = "i8x9"


def far_source_sha():
    h = hashlib.sha256()
    for f in ("far.hip", "far_lp.hip", "far_i8.hip", "far_common.h"):
        with open(os.path.join(ROOT, "paper_1710_01133_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec, blocking):
    """HBM bytes per far-field launch from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration);
    None when the kernel sources changed since the counters were taken, or
    when they were taken at another blocking (L, kchunk, max_split)."""
    path = os.path.join(ROOT, "profiles", "far_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    want = [blocking["block_L"], blocking["kchunk"], blocking["max_split"]]
    entries = t.get(prec) or []
    for e in entries if isinstance(entries, list) else [entries]:
        if e.get("source_sha") == far_source_sha() and e.get("blocking") == want:
            return e["bytes_per_launch"]
    return None


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM counters."""
    n = 1 << 28                                   # 2^28 floats = 1 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": True, "bytes_read_per_copy": 4 * n,
                      "bytes_written_per_copy": 4 * n, "copies": 3}))


def serving(abm, torch, inputs, n_req, arena_bytes, prec):
    """Open-loop Poisson stream (rate 200/s, seed 1710) of Duffing/Lorenz
    requests with their own alpha and N, served by the library's continuous
    batching loop; latency = completion seen by the server - submission."""
    reqs = inputs.serving_stream(n_req, far_prec=prec)
    ctx = abm.Context(0, arena_bytes=arena_bytes)
    ys = [abm.alloc_out(r.problem, 0) for r in reqs]
    tickets = [None] * n_req
    done = {}
    pending = set()
    i = 0
    t0 = time.perf_counter()
    while len(done) < n_req:
        now = time.perf_counter() - t0
        while i < n_req and reqs[i].arrival_s <= now:
            tickets[i] = abm.submit(ctx, reqs[i].problem, ys[i])
            pending.add(i)
            i += 1
        for j in list(pending):
            r = abm.poll(ctx, tickets[j])
            if r is not None:
                done[j] = r
                pending.discard(j)
        if time.perf_counter() - t0 > 600:
            raise RuntimeError("serving stream did not drain")
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    torch.cuda.synchronize()
    lat = np.array([done[j]["t_done"] - done[j]["t_submit"] for j in range(n_req)])
    queue = np.array([done[j]["t_start"] - done[j]["t_submit"] for j in range(n_req)])
    ok = sum(1 for j in range(n_req) if done[j]["status"] == 0)
    macs = sum(r.problem.history_macs() for r in reqs)
    # requests running at once (admitted, not yet done), sampled at every admission
    starts = np.array([done[j]["t_start"] for j in range(n_req)])
    ends = np.array([done[j]["t_done"] for j in range(n_req)])
    conc = [int(np.sum((starts <= t) & (ends > t))) for t in starts]
    # final states of the first 64 requests of the 2000-request stream (half
    # Lorenz, N up to 262144) against stored oracle runs: |y_N - oracle y_N|
    # over the oracle's max |y_s|, beside each request's noise floor (the
    # oracle's own change for x0 scaled by 1 + 1e-14)
    errs, floors = [], []
    path = os.path.join(ROOT, "tests", "golden", "serving_first64.json")
    if n_req == 2000 and os.path.exists(path):
        with open(path) as f:
            gold = json.load(f)
        for g in gold.values():
            j = g["index"]
            if done[j]["status"] == 0:
                y = ys[j].cpu().numpy()[-1]
                errs.append(float(np.max(np.abs(y - np.array(g["final"])))) / g["max_abs_y"])
                floors.append(g["noise_floor"])
    ctx.close()
    return {"requests": n_req, "ok": ok, "rate_per_s": 200.0, "arena_bytes": arena_bytes,
            "far_prec": prec, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "max_s": float(lat.max()),
            "p50_queue_s": float(np.percentile(queue, 50)),
            "p99_queue_s": float(np.percentile(queue, 99)),
            "mean_concurrent": float(np.mean(conc)), "max_concurrent": int(max(conc)),
            "max_rel_err_vs_oracle_final_state": max(errs) if errs else None,
            "median_rel_err_vs_oracle_final_state": float(np.median(errs)) if errs else None,
            "err_requests": len(errs),
            "err_requests_note": "the first 64 requests of the stream (Duffing and Lorenz, "
                                 "N up to 262144, fp32 far field); oracle noise floor of their "
                                 "final states up to %.2g" % max(floors) if floors else None,
            "wall_s": wall,
            "throughput_req_per_s": n_req / wall, "history_macs_per_s": macs / wall,
            "workload": "Poisson 200/s, half Duffing (d=2) half Lorenz (d=3), alpha~U[0.90,0.99], "
                        "N log-uniform [4096, 262144], h=2^-8, seed 1710"}


def normerr(y, ref):
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


def load_golden():
    """Stored oracle values (written by tests/golden/make_golden.py), or {}."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_fullsize.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def sweep_golden():
    """Stored oracle runs of all 1024 sweep members (every 1024th state,
    written by tests/golden/make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "duffing_sweep_all.npy")
    return np.load(path, allow_pickle=False) if os.path.exists(path) else None


def sweep_error(ys, gold):
    """Normwise error of every member against its stored oracle run: the max
    over all members, the member it occurs at, and the median."""
    if gold is None:
        return None
    e = np.array([normerr(y.cpu().numpy(), gold[i]) for i, y in enumerate(ys)])
    return {"max": float(e.max()), "argmax": int(e.argmax()), "median": float(np.median(e)),
            "members": int(e.size)}


def exclusive_far_rate(abm, ctx, probs, stride, tuning, prec):
    """The far-field kernel timed on its own: a plan whose far field and
    chains share one stream (no overlap between launches), per-launch HIP
    events on that stream."""
    os.environ["ABM_OVERLAP"] = "0"
    try:
        plan = abm.Plan(ctx, probs, out_stride=stride, tuning=tuning)
    finally:
        del os.environ["ABM_OVERLAP"]
    ys = [abm.alloc_out(p, stride) for p in probs]
    abm.solve_batch(plan, probs, ys)            # warm-up
    plan.timing(True)
    st = abm.solve_batch(plan, probs, ys)
    plan.timing(False)
    plan.check()
    plan.close()
    far_flop = 4.0 * st["far_macs"]
    achieved = far_flop / (st["far_ms"] / 1e3) / 1e12
    return {"achieved": achieved, "frac": achieved / PEAK_TFLOPS[prec],
            "executed_frac": achieved * EXEC_FACTOR[prec] / PEAK_TFLOPS[prec],
            "far_ms_total": st["far_ms"], "avg_launch_ms": st["far_ms"] / st["far_launches"],
            "chain_ms_total": st["chain_ms"], "launches": st["far_launches"]}


def time_batch(abm, torch, plan, probs, ys, steps, warmup):
    for _ in range(warmup):
        abm.solve_batch(plan, probs, ys)
    plan.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        st = abm.solve_batch(plan, probs, ys)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    plan.check()
    return dt, st


def small_batch_leg(abm, torch, inputs, ctx, steps=20):
    """A launch-bound batch (64 forced Duffing trajectories, N=8192, fp64 far
    field): the same solve launched eagerly and replayed from its graph."""
    probs = inputs.duffing_sweep(B=64, N=8192, far_prec="fp64")
    plan = abm.Plan(ctx, probs, out_stride=0)
    ys = [abm.alloc_out(p, 0) for p in probs]
    res = {"workload": "B=64 forced Duffing, alpha=0.95, h=2^-8, N=8192, d=2, far field fp64"}
    for mode in ("eager", "graph"):
        plan.graph(mode == "graph")
        dt, st = time_batch(abm, torch, plan, probs, ys, steps, 2)
        res[mode + "_ms"] = dt * 1e3
        res["launches"] = st["far_launches"] + st["chain_launches"]
    plan.close()
    return res


def cpu_baseline(inputs, budget_s=20.0):
    """The oracle as it stands on the host cores: a bounded sample of the
    sweep (whole trajectories at full N, OpenMP over trajectories)."""
    import oracle as O
    nthr = O.num_threads()
    sweep = inputs.duffing_sweep()
    # one trajectory takes ~5 s on one core: two per thread
    idx = list(range(2 * nthr))
    sample = [sweep[i] for i in idx]
    t0 = time.perf_counter()
    O.solve_batch([O.RHS_DUFFING] * len(sample), [p.alpha for p in sample],
                  [p.h for p in sample], [p.N for p in sample], [p.x0 for p in sample],
                  [p.p for p in sample], out_stride=0)
    dt = time.perf_counter() - t0
    macs = sum(p.history_macs() for p in sample)
    return {"value": macs / dt, "unit": "history MACs/s", "cores": nthr, "kind": "oracle",
            "sample": "%d of the 1024 sweep trajectories at full N=65536 (OpenMP over "
                      "trajectories), %.1f s wall" % (len(sample), dt)}


def plain_leg(abm, torch, inputs, ctx):
    """The plain per-step path (abm_solve) on the single 200000-step oscillator."""
    p1 = inputs.duffing_single()
    pp = abm.Plan(ctx, [p1], out_stride=0)
    y1 = abm.alloc_out(p1, 0)
    abm.solve(pp, p1, y1)
    pp.check()
    runs = []
    for _ in range(5):                       # median of 5 after one warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        abm.solve(pp, p1, y1)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t1)
    dt1 = float(np.median(runs))
    pp.check()
    pp.close()
    # algorithmic bytes if every step streamed its history and weights: per
    # (step, history index) the d history values and the two weights, 8 B each
    n = p1.N
    algo_bytes = n * (n + 1) / 2 * 8 * (p1.d + 2)
    res = {"workload": "forced Duffing, alpha=0.9, h=1e-3, N=200000, d=2, one trajectory",
           "seconds": dt1, "seconds_runs": runs, "history_macs_per_s": p1.history_macs() / dt1,
           "us_per_step": dt1 / p1.N * 1e6,
           "streamed_bytes": algo_bytes, "effective_GBps": algo_bytes / dt1 / 1e9,
           "frac_of_hbm_peak": algo_bytes / dt1 / 8e12,
           "note": "the history lives in LDS, so the bound is the per-step grid synchronisation"}
    # the scalar linear test (D^0.8 y = -y, N = 8192): plain path and the
    # blocked path on the same single trajectory (a narrow group)
    p0 = inputs.linear_c()
    pp = abm.Plan(ctx, [p0], out_stride=0)
    y0 = abm.alloc_out(p0, 0)
    times = {}
    for mode in ("plain", "blocked"):
        run = (lambda: abm.solve(pp, p0, y0)) if mode == "plain" else \
              (lambda: abm.solve_batch(pp, [p0], [y0]))
        run()
        pp.check()
        runs = []
        for _ in range(5):                   # median of 5
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t1)
        times[mode] = float(np.median(runs))
        pp.check()
    pp.close()
    res["linear_test"] = {"workload": "D^0.8 y = -y, y0 = 1, h = 2^-10, N = 8192, one trajectory",
                          "plain_us_per_step": times["plain"] / p0.N * 1e6,
                          "blocked_us_per_step": times["blocked"] / p0.N * 1e6}
    res["double_double"] = dd_leg(abm, torch, inputs, ctx,
                                  {"linear_N8192": (p0, times["plain"]),
                                   "oscillator_N200000": (p1, dt1)})
    return res


def dd_leg(abm, torch, inputs, ctx, cases):
    """The double-double mode (the counterpart of the paper's long-double
    runs) on the plain path's workloads: median of 3 after a warm-up, and its
    cost over the double plain path on the same problem."""
    res = {}
    for name, (p, t_double) in cases.items():
        q = inputs.Problem(p.rhs, p.alpha, p.h, p.N, p.x0, p.p, "dd", p.x1)
        plan = abm.Plan(ctx, [q], out_stride=0)
        y = abm.alloc_out(q, 0)
        abm.solve(plan, q, y)
        plan.check()
        runs = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            abm.solve(plan, q, y)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
        plan.check()
        plan.close()
        dt = float(np.median(runs))
        res[name] = {"seconds": dt, "seconds_runs": runs, "us_per_step": dt / p.N * 1e6,
                     "over_double_plain": dt / t_double}
    return res


def long_leg(abm, torch, inputs, ctx):
    """The paper's step counts (Table 1: 1e6 and 3e6 steps of one trajectory):
    the forced fractional LCR circuit (alpha = 0.9, h = 0.01, f = 0.117) by the
    blocked path, double far field; median of three solves after a warm-up."""
    res = {"workload": "forced fractional LCR circuit, alpha=0.9, h=0.01, f=0.117, d=2, "
                       "one trajectory, far field fp64",
           "paper_bgp_seconds": {"1000000": 69.06, "3000000": 304.17}}
    for N in (1000000, 3000000):
        p = inputs.Problem("LCR", 0.9, 0.01, N, (0.1, 0.0), inputs.LCR_P + (0.117,))
        plan = abm.Plan(ctx, [p], out_stride=0)
        y = abm.alloc_out(p, 0)
        abm.solve_batch(plan, [p], [y])      # warm-up
        runs = []
        for _ in range(3):                   # median of 3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            abm.solve_batch(plan, [p], [y])
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
        dt = float(np.median(runs))
        plan.check()
        plan.close()
        res[str(N)] = {"seconds": dt, "seconds_runs": runs,
                       "history_macs_per_s": p.history_macs() / dt, "us_per_step": dt / N * 1e6,
                       "parity": "tests/test_gpu_long.py: ~50 sampled steps of this launch "
                                 "shape recomputed by the oracle from the GPU's own states, "
                                 "each within its double-precision rounding bound"}
    return res


def lcr_leg(abm, torch, inputs, ctx, prec, tuning, steps=2):
    """The paper's own workload: the forced fractional LCR circuit swept over
    its forcing F in [0, 0.2] (B = 1024, N = 65536), commensurate orders
    (0.9, 0.9) as in its figures and incommensurate (0.9, 0.8), in the
    benchmark's far precision and in double, writing the
    stroboscopic (Poincare) section y(kT) (every 1142nd state, h = T/1142).
    Error against the stored oracle values (tests/golden) on the section
    points of the first 3600 steps of two members (the circuit is chaotic at
    some F, so later points measure the dynamics' amplification of rounding,
    not the method).  Reduced precisions run at the blocking chosen for the
    headline sweep (the same shape), double at the library's default."""
    gold = load_golden()
    M = inputs.LCR_SECTION_STEPS
    res = {"workload": "forced fractional LCR circuit, sigma=1.015, omega=0.55, a=-1.02, "
                       "b=-0.58, B=1024 forcings F in [0, 0.2], N=65536, h=T/1142, "
                       "Poincare section output (stride 1142)"}
    for al in ((0.9, 0.9), (0.9, 0.8)):
        for pr in (prec, "fp64"):
            probs = inputs.lcr_sweep(alpha=al, far_prec=pr)
            plan = abm.Plan(ctx, probs, out_stride=M, tuning=None if pr == "fp64" else tuning)
            plan.graph(True)
            ys = [abm.alloc_out(p, M) for p in probs]
            dt, st = time_batch(abm, torch, plan, probs, ys, steps, 1)
            errs = []
            for i in (300, 700):
                key = "lcr_sweep_%g_%g_%d" % (al[0], al[1], i)
                if key not in gold:
                    continue
                ref = np.array(gold[key]["y"])
                y = ys[i].cpu().numpy()[: ref.shape[0] - 1]
                errs.append(normerr(y, ref[:-1]))
            res["alpha=%s,%s %s" % (al[0], al[1], pr)] = {
                "ms_per_step": dt * 1e3, "history_macs_per_s": st["history_macs"] / dt,
                "section_points_per_member": int(ys[0].shape[0]), "blocking": plan.config(),
                "max_rel_err_vs_oracle_first_3600_steps": max(errs) if errs else None}
            plan.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default=DEFAULT_PREC, choices=list(PEAK_TFLOPS))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-only", action="store_true",
                    help="only the plain per-step path on the 200000-step oscillator")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving stream (0 skips the serving leg)")
    ap.add_argument("--serve-arena-mib", type=int, nargs="+", default=[96, 8192],
                    help="arena sizes to serve the stream with (the first binds admission)")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the sweep at the other far-field precisions")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-lcr", action="store_true",
                    help="skip the LCR forcing sweep (the paper's workload)")
    ap.add_argument("--no-long", action="store_true",
                    help="skip the 1e6 / 3e6-step single-trajectory runs")
    ap.add_argument("--tune-budget", type=float, default=20.0,
                    help="seconds for the autotuner to choose the blocking (0: library defaults)")
    ap.add_argument("--blocking", default=None,
                    help="L,kchunk,max_split: use this blocking instead of autotuning")
    ap.add_argument("--eager", action="store_true",
                    help="launch the batched solve eagerly instead of replaying its captured graph")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the batched sweep is sized for one MI355X and no "
              "multi-GPU path is built (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_01133_amd import abm, inputs
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    ctx = abm.Context(0)
    if args.plain_only:
        print(json.dumps({"plain": plain_leg(abm, torch, inputs, ctx)}))
        ctx.close()
        return

    stride = 1024
    probs = inputs.duffing_sweep(far_prec=args.prec)
    # blocking chosen by the library's autotuner (whole solves of this sweep)
    tuning = None
    tune_report = None
    if args.blocking:
        Lb, kb, sb = (int(x) for x in args.blocking.split(","))
        tuning = {"block_L": Lb, "kchunk": kb, "max_split": sb, "column_tiles_only": 0}
    elif args.tune_budget > 0:
        t0 = time.perf_counter()
        best, trials = abm.autotune(ctx, probs, out_stride=stride, budget_s=args.tune_budget)
        tuning = best
        tune_report = {"best": best, "seconds": time.perf_counter() - t0,
                       "trials": [{"cfg": t["cfg"], "ms": round(t["ms"], 2), "status": t["status"]}
                                  for t in trials]}
    t0 = time.perf_counter()
    plan = abm.Plan(ctx, probs, out_stride=stride, tuning=tuning)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    ys = [abm.alloc_out(p, stride) for p in probs]
    plan.graph(not args.eager)
    dt, st = time_batch(abm, torch, plan, probs, ys, args.steps, args.warmup)
    macs = st["history_macs"]
    value = macs / dt
    eager_dt = None
    if not args.eager:                      # the same solve launched eagerly, for comparison
        plan.graph(False)
        eager_dt, _ = time_batch(abm, torch, plan, probs, ys, args.steps, 1)
        plan.graph(True)

    # error of every member against the stored double-precision oracle runs
    gold = sweep_golden()
    errs = sweep_error(ys, gold)
    max_err = errs["max"] if errs else None

    # roofline of the far-field kernel: one more solve with per-launch events
    plan.timing(True)
    stt = abm.solve_batch(plan, probs, ys)
    plan.timing(False)
    plan.check()
    far_flop = 4.0 * stt["far_macs"]          # predictor + corrector multiply-add per history MAC
    far_s = stt["far_ms"] / 1e3
    achieved = far_flop / far_s / 1e12
    peak = PEAK_TFLOPS[args.prec]
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(args.prec, plan.config()),
            "kernel": "far-field Toeplitz x history product (%s)" % args.prec,
            "launches": stt["far_launches"], "avg_launch_ms": stt["far_ms"] / stt["far_launches"],
            "flop_per_launch": far_flop / stt["far_launches"],
            "executed_frac": achieved * EXEC_FACTOR[args.prec] / peak,
            "chain_ms_total": stt["chain_ms"], "far_ms_total": stt["far_ms"],
            # launches of consecutive ticks overlap: the far field's rate over
            # the whole solve's wall time, for comparison
            "achieved_over_solve_wall": far_flop / dt / 1e12}
    # the far-field kernel on its own (launches serialised on one stream):
    # the kernel's own rate, reported as achieved/frac; the overlapped
    # per-launch figure and the solve-wall bound are kept beside it
    excl = exclusive_far_rate(abm, ctx, probs, stride, plan.config(), args.prec)
    roof["overlapped"] = {"achieved": roof["achieved"], "frac": roof["frac"],
                          "avg_launch_ms": roof["avg_launch_ms"]}
    roof["achieved"] = excl["achieved"]
    roof["frac"] = excl["frac"]
    roof["executed_frac"] = excl["executed_frac"]
    roof["avg_launch_ms"] = excl["avg_launch_ms"]
    roof["exclusive"] = excl
    roof["measure"] = ("achieved/frac: useful FLOP (4 per far-field history MAC) over the far "
                       "kernel's own launch time, launches serialised on one stream; "
                       "overlapped: the same launches timed inside the overlapped solve")

    plain = None if args.no_plain else plain_leg(abm, torch, inputs, ctx)
    longrun = None if args.no_long else long_leg(abm, torch, inputs, ctx)
    lcr = None if args.no_lcr else lcr_leg(abm, torch, inputs, ctx, args.prec, plan.config())
    small = small_batch_leg(abm, torch, inputs, ctx)

    serve = None
    if args.serve_requests > 0:
        serve = {"arena_%dMiB" % mib: serving(abm, torch, inputs, args.serve_requests, mib << 20,
                                              "fp32")
                 for mib in args.serve_arena_mib}

    # the same sweep at the other far-field precisions (error against the same oracle runs)
    others = None
    if not args.no_precisions:
        others = {}
        for pr in ("fp64", "fp32", "bf16x6", "i8x9", "fp16x3", "bf16x3"):
            if pr == args.prec:
                continue
            pp = inputs.duffing_sweep(far_prec=pr)
            # reduced precisions at the headline's blocking, double at the default
            pl2 = abm.Plan(ctx, pp, out_stride=stride, tuning=None if pr == "fp64" else plan.config())
            pl2.graph(not args.eager)
            dt2, st2 = time_batch(abm, torch, pl2, pp, ys, 2, 1)
            e2 = sweep_error(ys, gold)
            others[pr] = {"value": st2["history_macs"] / dt2, "ms_per_step": dt2 * 1e3,
                          "blocking": pl2.config(),
                          "max_rel_err_vs_oracle": e2["max"] if e2 else None,
                          "err_all_members": e2}
            pl2.close()

    cpu = None if args.no_cpu else cpu_baseline(inputs)

    out = {
        "metric": "history MACs/s (d*N(N+1)/2 per trajectory), batched sweep",
        "value": value,
        "unit": "history MACs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded forcing sweep)",
        "config": {"workload": "forcing sweep: B=1024 forced Duffing, alpha=0.95, h=2^-8, "
                               "N=65536, d=2, far field %s" % args.prec,
                   "B": 1024, "N": 65536, "d": 2, "block_L": st["block_L"],
                   "blocking": plan.config(),
                   "far_prec": args.prec, "launch": "eager" if args.eager else "graph"},
        "eager_ms_per_step": None if eager_dt is None else eager_dt * 1e3,
        "launch_bound_batch": small,
        "long_trajectory": longrun,
        "lcr_sweep": lcr,
        "max_rel_err_vs_oracle": max_err,
        "err_all_members": errs,
        "plan_seconds": plan_s,
        "autotune": tune_report,
        "roofline": roof,
        "plain": plain,
        "batched_over_plain": (value / plain["history_macs_per_s"]) if plain else None,
        "serving": serve,
        "other_precisions": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
