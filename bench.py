#!/usr/bin/env python3
"""Benchmark of the MI355X lot-sizing VNS: exact move-evaluations per second, and time to the plain
method's best cost, learned vs plain.

Workload (default): the learned + batched set, 1024 synthetic instances with K ~ U{100..1000} products and
T in {52, 104} periods (demand U{0..200}, returns floor(D * U(0.1, 0.9)), setup costs U{200..2000}, holding
hM U{2..6}, hR U{1..hM}; instance i drawn from SeedSequence([5, i])), 16 Philox chains each: 16,384 chains,
~2.8e9 move slots per full sweep, all resident in HBM.  It is the largest workload that fits one GPU.

One step = one exact sweep: every move of the neighbourhoods flip zM, flip zR and shift for every chain
(the pricing kernel k_eval), followed by each chain's lexicographic (price, slot) argmin (k_chain_best),
whose results are copied to the host.  The sweeps run on the states the plain GVNS search reached after the
workload's 5000 iterations (local optima, as in the VND's last passes).  `value` = move-evaluations of the
K timed steps / their device time (HIP events on the stream the kernels run on); inputs are resident before
the timed region starts.

Beside it, on the same GPU in the same run:
  * `time_to_plain_best`: the plain search runs the workload's 5000 iterations (launches of --chunk); per
    instance its best cost over the chains is the target.  The learned search (a scorer trained on moves the
    search logged on 16 disjoint instances ranks each neighbourhood's moves, the best-ranked 10% are priced
    exactly, the whole neighbourhood when none of them improves) runs on the same instances, seeds and chains
    until every instance reaches its target.  Device times of both, the scorer's and the training's rates.
  * `search`: the plain GVNS search's exact move-evaluations/s over the configured iterations: the 100 x 52
    instance with 64 chains x 2000 iterations in one launch (with its kernel's roofline), the 4096-instance
    batch with 8 chains x 1000 iterations in one launch, and the 1024-instance set's 5000 iterations.
  * `sweeps`: the same step on the 4096-instance batch (8 chains, after its 1000 iterations) and on the
    100 x 52 instance (64 chains, after its 2000 iterations).
  * `time_to_plain_best_100x52`: the same comparison on the 100 x 52 instance (64 chains, 2000 iterations).
  * `cpu_baseline`: the CPU oracle's exact sweep (every move of the three neighbourhoods priced by its
    look-ahead decode) on a sample of the workload's instances, one thread and every host thread.
  * `paper_quality`: a Table-1-shaped comparison on the paper's benchmark shape (108 synthetic instances of
    300 x 52): GVNS, best-of-4 in both forms and the learned search, the same device time each; the CPU leg
    adds the oracle's serial VND from the initial solution.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU peak of MI355X for the decode's own operation mix, from unit counts and clock: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 39.3e12 lane-slots/s.  Of the 14 operations of a period-step, 10 (bfe x2, bfi x4, min,
# mad x2, and_or) take a lane-slot each and 4 (add, sub x2, the bitop3 of the no-setup mask) take half of one:
# gfx950 issues that class at twice the rate (the probe in csrc/valu_probe.hip, `bench.py --valu-probe`).
# 12 lane-slots per period-step make the peak 3.28e12 period-steps/s, 45.9e12 of these operations per second.
OPS_PER_PERIOD_STEP = 14     # operations of one period-step of the forward decode
LANE_SLOTS_PER_STEP = 12
CU, SIMD_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
VALU_PEAK_OPS = CU * SIMD_PER_CU * LANES_PER_SIMD * CLOCK_HZ * OPS_PER_PERIOD_STEP / LANE_SLOTS_PER_STEP
TUNE_FILE = os.path.join(ROOT, "paper_1704_05132_amd", "tune_table.json")
BEST_OF_G = 4                # best-of-G search (Algorithm 2) measured beside the plain one: shakes per iteration
LEARNED_SPEC_M = 8           # speculative iterations of the learned search (4 wavefronts per workgroup)
PACKED_P, PACKED_WAVES = 8, 2   # the packed learned search's batch and workgroup (its fastest measured shape)
# learned scorer: 2 x (16*64 + 64*64 + 64) flops per scored move; dense bfloat16 matrix-core peak of MI355X
MLP_FLOP_PER_ROW = 2 * (16 * 64 + 64 * 64 + 64)
BF16_PEAK_TFLOPS = 2500.0
METRIC = "exact move-evals/s (int64 cost) + time-to-plain-best-cost, learned vs plain"
SWEEP_LAUNCH = ("k_eval: every chain, neighbourhoods flip zM + flip zR + shift, tuned launch shape (chains per "
                "workgroup, or pair ranges spread over the compute units)")
SEARCH_LAUNCH = "search: every chain, the workload's iterations in one launch, tuned launch shape"


def kernel_source_hash():
    """sha256 over the HIP sources: counter-based traffic is reported only for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1704_05132_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, launch):
    """HBM bytes per launch of `kernel` in `launch` on `workload`, from the committed rocprofv3 counter summary
    (profiles/traffic_<workload>.json), if it was taken on the current kernels."""
    try:
        with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = t.get("launches", {}).get(launch, {}).get(kernel)
    return None if e is None else e["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="learned_batched_1024",
                    choices=["learned_batched_1024", "batched_4096", "plain_100x52", "paper_300x52"])
    ap.add_argument("--steps", type=int, default=20, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=5, help="untimed sweeps before them")
    ap.add_argument("--search-iters", type=int, default=None,
                    help="iterations of the searches (default: the workload's own, 5000 / 1000 / 2000)")
    ap.add_argument("--only-sweep", action="store_true",
                    help="only the workload's search, as one launch, and the timed sweeps (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain time-to-best halves")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="target time of each oracle sample")
    ap.add_argument("--chunk", type=int, default=50, help="iterations per launch in the time-to-best runs")
    ap.add_argument("--learned-permille", type=int, default=100, help="share of moves priced exactly (1/1000)")
    ap.add_argument("--learned-pack", type=int, default=0,
                    help="learned VND: products per wavefront batch (packed form; 0 = one product at a time)")
    ap.add_argument("--no-packed-leg", dest="packed_leg", action="store_false",
                    help="skip the packed learned search on the batched set")
    ap.add_argument("--learned-waves", type=int, default=0,
                    help="learned search: wavefronts per workgroup (0 = the tuned plain search's)")
    ap.add_argument("--learned-log-iters", type=int, default=200)
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--quality-ms", type=float, default=1000.0,
                    help="device time each search arm of the Table-1-shaped comparison gets")
    ap.add_argument("--no-quality", action="store_true", help="skip the Table-1-shaped comparison on 300 x 52")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration for profiling runs)")
    ap.add_argument("--valu-probe", action="store_true", help="run the VALU issue-rate probe and print its JSON")
    ap.add_argument("--print-source-hash", action="store_true")
    return ap.parse_args()


# ---------------------------------------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------------------------------------
def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def new_ctx(vns, insts, w, stream, table, key, chains=None, trace=False, options=None):
    """A context on the workload's instances with the tuned launch shape, then `options` over it."""
    target = insts[0] if len(insts) == 1 else insts
    c = vns.Context(target, seed=w["seed"], chains=chains or w["chains"], nb_list=w["nb"], trace=trace)
    c.bind_stream(stream)
    table.apply(c, key)
    for opt, v in (options or {}).items():
        c.set_option(opt, v)
    return c


def sweep_steps(torch, vns, ctx, stream, steps, warmup):
    """`warmup` untimed, then `steps` timed exact sweeps of every chain (one step: pricing kernel, per-chain
    argmin, results to the host).  Device time of the steps from HIP events on the stream, the pricing
    kernel's own time per step from the library's events around it."""
    for _ in range(warmup):
        ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False, prod_best=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k_ms, evals, psteps = [], 0, 0
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False, prod_best=False)
        s = ctx.stats()
        k_ms.append(s["last_eval_ms"])
        evals += s["last_eval_evals"]
        psteps += s["last_eval_period_steps"]
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    achieved = psteps * OPS_PER_PERIOD_STEP / (sum(k_ms) / 1e3) / 1e12
    wide = ctx.get_option(vns.OPT_EVAL_SPREAD) > 4   # the range form with 8-16 wavefronts per workgroup
    return {"steps": steps, "move_evals_per_step": evals // max(steps, 1), "device_ms": ms, "wall_s": wall,
            "value": evals / (ms / 1e3), "unit": "move-evals/s", "kernel": "k_eval_wide" if wide else "k_eval",
            "launch_shape": {"spread": ctx.get_option(vns.OPT_EVAL_SPREAD),
                             "group": ctx.get_option(vns.OPT_EVAL_GROUP)},
            "kernel_ms_mean": sum(k_ms) / len(k_ms), "kernel_ms_median": statistics.median(k_ms),
            "kernel_share": sum(k_ms) / ms, "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12,
            "frac": achieved / (VALU_PEAK_OPS / 1e12)}


def warm_search(vns, make_ctx):
    """A few iterations on a throwaway context of the same launch shape.  The first cooperative launch in a
    process waits for the runtime's one-time set-up (a 4.5 ms gap before the kernel starts on the 100 x 52
    launch), which the library's events would otherwise count as search time."""
    c = make_ctx()
    c.run(4)
    c.close()


def search_once(vns, ctx, iters):
    """One launch of `iters` GVNS iterations of every chain; the search kernel's rate and roofline (the
    evaluations the search consumed; speculative iterations thrown away are counted apart)."""
    ctx.run(iters)
    st = ctx.stats()
    ms, evals = st["last_run_ms"], st["last_run_evals"]
    spec_m, discarded = st["last_run_spec_iters"], st["last_run_discarded_evals"]
    achieved = st["last_run_period_steps"] * OPS_PER_PERIOD_STEP / (ms / 1e3) / 1e12
    executed = (evals + discarded) / evals if evals else 1.0
    best = ctx.get_option(vns.OPT_BEST_OF)
    return {"iters": iters, "kernel": "k_run_coop" if spec_m > 1 or best > 1 else "k_run", "kernel_ms": ms,
            "move_evals": evals, "value": evals / (ms / 1e3), "unit": "move-evals/s",
            "iterations_per_s": iters / (ms / 1e3), "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12,
            "unit_achieved": "TOP/s", "frac": achieved / (VALU_PEAK_OPS / 1e12),
            "speculative_iterations": spec_m, "discarded_move_evals": discarded,
            "executed_over_consumed": executed, "executed_frac": achieved * executed / (VALU_PEAK_OPS / 1e12)}


def chunked_search(make_ctx, n_inst, chains, max_iters, chunk, targets=None, horizon_ms=None, keep=False):
    """Run a fresh context in launches of `chunk` iterations.  Per instance, the best cost over its chains
    is tracked after every launch.  Stops once every instance is at or below `targets` (when given).
    Returns the device ms and iterations at which all targets were reached (None if not), the final
    per-instance bests, the total device ms and evaluations, the per-launch history (ms, iterations, bests),
    and the share of instances at their target when the device time first reached `horizon_ms`.  With `keep`
    the context is returned open under "ctx"."""
    import numpy as np
    ctx = make_ctx()
    ms, it, evals, reached, hist, share_at = 0.0, 0, 0, None, [], None
    nb_evals, fallbacks, discarded = 0, 0, 0
    best = ctx.costs()[1].reshape(n_inst, chains).min(1)
    while it < max_iters:
        n = min(chunk, max_iters - it)
        ctx.run(n)
        st = ctx.stats()
        ms += st["last_run_ms"]
        evals += st["last_run_evals"]
        nb_evals += st["last_run_learned_evals"]
        fallbacks += st["last_run_fallbacks"]
        discarded += st["last_run_discarded_evals"]
        it += n
        best = ctx.costs()[1].reshape(n_inst, chains).min(1)
        hist.append((ms, it, best.copy()))
        if targets is not None:
            if horizon_ms is not None and share_at is None and ms >= horizon_ms:
                share_at = float(np.mean(best <= targets))
            if (best <= targets).all():
                reached = (ms, it)
                break
    out = {"ms": reached[0] if reached else None, "iters": reached[1] if reached else it, "best": best,
           "total_ms": ms, "total_iters": it, "evals": evals, "hist": hist, "share_at_horizon": share_at,
           "nb_evals": nb_evals, "fallbacks": fallbacks, "discarded": discarded}
    if keep:
        out["ctx"] = ctx
    else:
        ctx.close()
    return out


LEARNED_SETUP = {
    # evaluation workload -> (training workload, first training index, training instances, chains while logging)
    "plain_100x52": ("learned_100x52", 100, 16, 16),
    "learned_batched_1024": ("learned_batched_1024", 4096, 16, 4),
}


def learned_vs_plain(args, vns, stream, table, key, name, insts, w, plain):
    """Time to the plain method's best cost, per instance: the plain search (`plain`, a chunked_search run over
    the workload's iterations) vs the learned search (scorer trained on moves the search logged on disjoint
    training instances), same instances, seeds and chains, this GPU."""
    import numpy as np
    from paper_1704_05132_amd.instances import workload
    n_inst, chains, chunk, iters = len(insts), w["chains"], args.chunk, plain["total_iters"]

    def make(options=None):
        return new_ctx(vns, insts, w, stream, table, key, options=options)

    B = plain["best"]
    first = next(h for h in plain["hist"] if (h[2] <= B).all())
    plain_ms, plain_it = first[0], first[1]

    # training set: moves logged by the search on disjoint instances
    tw, t0i, n_train, log_chains = LEARNED_SETUP[name]
    train = [workload(tw, t0i + j) for j in range(n_train)]
    t0 = time.perf_counter()
    with vns.Context(train, seed=w["seed"], chains=log_chains, nb_list=w["nb"], trace=False,
                     options={vns.OPT_LOG: 2_000_000}) as lg:
        lg.bind_stream(stream)
        lg.run(args.learned_log_iters)
        log_ms = lg.stats()["last_run_ms"]
        X, y = lg.move_log()
    with make() as tr:
        tr.mlp_init(7)
        t1 = time.perf_counter()
        loss = tr.mlp_train(X, y, epochs=args.learned_epochs, batch=4096, lr=2e-3, seed=11)
        train_s = time.perf_counter() - t1
        st = tr.stats()
        train_dev_ms, train_rows = st["last_mlp_ms"], st["last_mlp_rows"]
        params = tr.mlp_get()
        # scorer alone: one launch over 2^20 feature rows (the logged moves, repeated)
        Xs = np.resize(X, (1 << 20, X.shape[1])) if len(X) else np.zeros((1 << 20, 16), np.float32)
        for _ in range(3):
            tr.mlp_score(Xs)
        st = tr.stats()
        score_ms, score_rows = st["last_mlp_ms"], st["last_mlp_rows"]
    collect_s = time.perf_counter() - t0 - train_s

    def make_learned():
        c = make({vns.OPT_LEARNED: args.learned_permille, vns.OPT_LEARNED_PACK: args.learned_pack})
        if c.get_option(vns.OPT_SPEC_ITERS) > 1:
            # the learned kernel keeps the scorer's weights in registers (about 250 VGPRs, two wavefronts per
            # SIMD), so its speculative launch takes two 4-wavefront workgroups per compute unit
            c.set_option(vns.OPT_RUN_WAVES, 4)
            c.set_option(vns.OPT_SPEC_ITERS, LEARNED_SPEC_M)
        if args.learned_waves:
            c.set_option(vns.OPT_RUN_WAVES, args.learned_waves)
        c.mlp_set(params)
        return c

    lrn = chunked_search(make_learned, n_inst, chains, 2 * iters, chunk, targets=B, horizon_ms=plain["total_ms"])
    if lrn["share_at_horizon"] is None:   # reached (or stopped) before the plain run's total time
        lrn["share_at_horizon"] = float(np.mean(lrn["best"] <= B))
    packed = None
    if args.packed_leg and n_inst > 1 and not args.learned_pack:
        # the packed form of the same learned search (VNS_OPT_LEARNED_PACK): same moves, its own time
        def make_packed():
            c = make({vns.OPT_LEARNED: args.learned_permille, vns.OPT_LEARNED_PACK: PACKED_P,
                      vns.OPT_RUN_WAVES: PACKED_WAVES})
            c.mlp_set(params)
            return c
        pk = chunked_search(make_packed, n_inst, chains, 2 * iters, chunk, targets=B)
        packed = {"products_per_wavefront": PACKED_P, "waves": PACKED_WAVES, "ms_to_plain_best": pk["ms"],
                  "iters": pk["iters"], "speedup": (plain_ms / pk["ms"]) if pk["ms"] else None,
                  "device_us_per_chain_iteration": pk["total_ms"] * 1e3 / max(pk["total_iters"], 1),
                  "reason": "the shared selection and fallback passes save about a quarter of the wavefront "
                            "passes, and the lockstep's workgroup barriers and per-product serial steps (state, "
                            "move lists, scoring) cost about as much"}
    out = {
        "instances": n_inst, "chains": chains, "iters": iters, "chunk_iters": chunk,
        "plain_ms_to_best": plain_ms, "plain_iters_to_best": plain_it, "plain_total_ms": plain["total_ms"],
        "learned_ms_to_plain_best": lrn["ms"], "learned_iters": lrn["iters"], "learned_reached": lrn["ms"] is not None,
        "learned_share_at_plain_total_ms": lrn["share_at_horizon"],
        "speedup": (plain_ms / lrn["ms"]) if lrn["ms"] else None,
        "permille_priced": args.learned_permille, "learned_pack": args.learned_pack,
        "training": {"instances": len(train), "logged_moves": int(len(y)),
                     "improving_share": float(np.mean(y < 0)) if len(y) else 0.0,
                     "log_search_ms": log_ms, "collect_s": collect_s, "epochs": args.learned_epochs,
                     "train_s": train_s, "final_loss": loss, "device_ms": train_dev_ms,
                     "rows_per_s": train_rows / (train_dev_ms / 1e3) if train_dev_ms else None,
                     "tflops": (train_rows * 3 * MLP_FLOP_PER_ROW / (train_dev_ms / 1e3) / 1e12
                                if train_dev_ms else None)},
        "scorer": {"kernel": "k_mlp_score", "rows": score_rows, "ms": score_ms,
                   "rows_per_s": score_rows / (score_ms / 1e3), "bound": "mfma",
                   "achieved": score_rows * MLP_FLOP_PER_ROW / (score_ms / 1e3) / 1e12, "peak": BF16_PEAK_TFLOPS,
                   "unit": "TFLOP/s",
                   "frac": score_rows * MLP_FLOP_PER_ROW / (score_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS,
                   "flop_per_row": MLP_FLOP_PER_ROW,
                   # its bytes: a 64-byte float32 feature row in, a 4-byte score out (152 flops per byte, under
                   # the 312 at which the matrix cores and HBM balance, so HBM is the lower roof)
                   "hbm_GBps": score_rows * 68 / (score_ms / 1e3) / 1e9, "hbm_frac": score_rows * 68 / (score_ms / 1e3) / 8e12},
        "note": "device time of the search launches only; scorer training is reported separately",
    }
    # where the time goes, per GVNS iteration of every chain (whole runs, chunked as above)
    n_ch = n_inst * chains

    def per_it(r):
        its = max(r["total_iters"], 1) * n_ch
        d = {"device_us_per_chain_iteration": r["total_ms"] * 1e3 / max(r["total_iters"], 1),
             "exact_evals": r["evals"] / its, "discarded_evals": r["discarded"] / its}
        if r["nb_evals"]:
            d["neighbourhood_evals"] = r["nb_evals"] / its
            d["fallback_share"] = r["fallbacks"] / r["nb_evals"]
        return d
    out["per_iteration"] = {"plain": per_it(plain), "learned": per_it(lrn)}
    if packed is not None:
        out["packed"] = packed
    out["reason"] = ("a learned neighbourhood evaluation scores every move (MFMA) and then needs the exact prices "
                     "of the best-ranked share, with one move per lane over all T periods (the same decode latency "
                     "as pricing the whole neighbourhood), and of the whole neighbourhood when none of them "
                     "improves (fallback_share; both come from one pricing when the neighbourhood fits two "
                     "wavefront passes); exact pricing runs near the int32 peak, so fewer exact evaluations do not "
                     "buy back the scoring and the fallbacks")
    if n_inst == 1:
        out["plain_best_F"] = int(B[0])
        out["learned_best_F"] = int(lrn["best"][0])
    else:
        out["plain_best_F_sum"] = int(B.sum())
        out["learned_best_F_sum"] = int(lrn["best"].sum())
    return out


def cpu_baseline(insts, w, name, target_s):
    """The oracle as it is, on this host: its exact sweep (orc_price_all, every move of the three
    neighbourhoods) of random feasible setup patterns of the workload's instances, first on one thread, then
    one instance per thread on every host thread (up to 16).  Each sample is sized to about target_s."""
    import numpy as np
    import oracle
    from paper_1704_05132_amd.instances import random_pattern
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(insts))
    nthreads = host_threads()

    def one(i, reps, seed):
        inst = insts[i]
        zM, zR = random_pattern(inst, np.random.default_rng(seed))
        n = 0
        for _ in range(reps):
            n += oracle.price_all(inst, zM, zR, 7)[1]
        return n

    # one thread: instances in the sampled order until target_s has passed
    t0, n1, used = time.perf_counter(), 0, 0
    while time.perf_counter() - t0 < target_s and used < len(order):
        n1 += one(int(order[used]), 1, used)
        used += 1
    dt1 = time.perf_counter() - t0
    rate1 = n1 / dt1
    # every thread: one instance each, repeated so that each thread runs about target_s
    per_sweep = dt1 / max(used, 1)
    reps = max(1, int(target_s / max(per_sweep, 1e-6)))
    picks = [int(order[j % len(order)]) for j in range(nthreads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        nN = sum(ex.map(lambda a: one(a[1], reps, 1000 + a[0]), enumerate(picks)))
    dtN = time.perf_counter() - t0
    Ks = [insts[i].K for i in picks]
    return {"value": nN / dtN, "unit": "move-evals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"oracle exact sweeps (flip zM, flip zR, shift) of random feasible patterns of {name} "
                      f"instances: {nthreads} threads x {reps} sweeps of one instance each (K {min(Ks)}..{max(Ks)}), "
                      f"{nN} move-evaluations in {dtN:.1f} s",
            "single_thread": {"value": rate1, "instances": used, "move_evals": n1, "seconds": dt1},
            "nproc": os.cpu_count(), "threads_available": nthreads, "cpu_model": cpu_model()}


def valu_probe():
    """Issue rates of the decode's integer operations (csrc/valu_probe.hip), as lane-operations per CU per
    nominal 2.4 GHz clock, and the decode step's rate as period-steps and operations per second."""
    import ctypes
    import torch  # noqa: F401  (one HIP runtime in the process)
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1704_05132_amd", "libvaluprobe.so"))
    L.valu_probe_name.restype = ctypes.c_char_p
    L.valu_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
    grid, iters = 8192, 4096     # 4-wave workgroups: 32 waves per SIMD over the run, 8 resident at a time
    out = {"grid_workgroups": grid, "workgroup": 256, "iters": iters, "clock_hz": CLOCK_HZ, "cu": CU, "ops": {}}
    for op in range(L.valu_probe_count()):
        best = None
        for _ in range(3):
            ms, n = ctypes.c_double(), ctypes.c_double()
            rc = L.valu_probe_run(op, grid, iters, ctypes.byref(ms), ctypes.byref(n))
            if rc != 0:
                raise RuntimeError(f"valu probe {op} failed: hip error {rc}")
            best = ms.value if best is None else min(best, ms.value)
        per_cu_clk = n.value / (best / 1e3) / CU / CLOCK_HZ
        nm = L.valu_probe_name(op).decode()
        out["ops"][nm] = {"ms": best, "lane_ops": n.value, "lane_ops_per_cu_per_clock": per_cu_clk}
        if nm == "decode_step":
            out["ops"][nm]["period_steps_per_s"] = n.value / (best / 1e3)
            out["ops"][nm]["ops_per_s"] = n.value / (best / 1e3) * OPS_PER_PERIOD_STEP
            out["ops"][nm]["frac_of_derived_peak"] = n.value / (best / 1e3) * OPS_PER_PERIOD_STEP / VALU_PEAK_OPS
    out["derived_peak_ops_per_s"] = VALU_PEAK_OPS
    return out


def paper_quality(args, vns, stream):
    """A table shaped like the paper's Table 1 on its benchmark shape (synthetic: 108 instances of 300
    products x 52 periods): every search gets the same device time on all instances at once, with 8
    workgroups per instance, and the best cost per instance is compared across searches.  The serial VND arm
    (the oracle on the host) is added by the CPU-baseline leg, serial_vnd_arm."""
    import numpy as np
    from paper_1704_05132_amd.instances import workload
    w, insts = workload_insts("paper_300x52")
    n, seed, nb = len(insts), w["seed"], w["nb"]

    def ctx_of(chains, options):
        c = vns.Context(insts, seed=seed, chains=chains, nb_list=nb, trace=False, options=options)
        c.bind_stream(stream)
        return c

    def run_for(make_ctx, chains):
        ctx = make_ctx()
        ms, it = 0.0, 0
        while ms < args.quality_ms:
            ctx.run(args.chunk)
            ms += ctx.stats()["last_run_ms"]
            it += args.chunk
        best = ctx.costs()[1].reshape(n, chains).min(1)
        ctx.close()
        return best, ms, it

    arms = {}
    arms["gvns"] = (run_for(lambda: ctx_of(8, {vns.OPT_RUN_WAVES: 2}), 8), 8, 1)
    arms["best_of_4"] = (run_for(lambda: ctx_of(2, {vns.OPT_BEST_OF: 4, vns.OPT_RUN_WAVES: 2}), 2), 2, 4)
    arms["best_of_4_literal"] = (run_for(lambda: ctx_of(2, {vns.OPT_BEST_OF: 4, vns.OPT_BEST_OF_LITERAL: 1,
                                                            vns.OPT_RUN_WAVES: 2}), 2), 2, 4)
    # learned: a scorer trained on moves the search logged on 8 disjoint instances of the same shape
    train = [workload("paper_300x52", 1000 + j) for j in range(8)]
    with vns.Context(train, seed=seed, chains=2, nb_list=nb, trace=False, options={vns.OPT_LOG: 2_000_000}) as lg:
        lg.bind_stream(stream)
        lg.run(100)
        X, y = lg.move_log()
    with ctx_of(1, None) as tr:
        tr.mlp_init(7)
        tr.mlp_train(X, y, epochs=args.learned_epochs, batch=4096, lr=2e-3, seed=11)
        params = tr.mlp_get()

    def make_learned():
        c = ctx_of(8, {vns.OPT_LEARNED: args.learned_permille, vns.OPT_RUN_WAVES: args.learned_waves or 2,
                       vns.OPT_LEARNED_PACK: args.learned_pack})
        c.mlp_set(params)
        return c

    arms["learned"] = (run_for(make_learned, 8), 8, 1)
    table = np.stack([r[0] for r, _, _ in arms.values()])
    best = table.min(0)
    paper_quality.best_per_instance = best   # the serial VND arm's gaps are measured against it
    out = {"instances": n, "K": insts[0].K, "T": insts[0].T, "device_ms_per_search": args.quality_ms,
           "chunk_iters": args.chunk, "logged_moves": int(len(y)), "note": "best cost per instance after the same "
           "device time; best_on counts the instances where a search holds the lowest cost (ties count for each)"}
    for i, (a, ((_, ms, it), chains, streams)) in enumerate(arms.items()):
        out[a] = {"mean_best_F": float(table[i].mean()), "best_on": int((table[i] == best).sum()),
                  "mean_gap_pct": float(((table[i] - best) / best).mean() * 100), "iterations": it, "device_ms": ms,
                  "chains_per_instance": chains, "streams": streams}
    return out


def serial_vnd_arm(target_best):
    """The serial VND arm of the Table-1-shaped comparison (the paper's serial baseline): the oracle's VND
    (Algorithm 1, every product in every pass) from the initial solution zM = 1, zR = 0 on each of the 108
    instances, one instance per host thread; its cost against the best the device searches reached."""
    import numpy as np
    import oracle
    w, insts = workload_insts("paper_300x52")
    nthreads = host_threads()

    def one(inst):
        t0 = time.perf_counter()
        F, _, _, ev = oracle.vnd(inst, np.ones((inst.K, inst.T), np.uint8), np.zeros((inst.K, inst.T), np.uint8),
                                 w["nb"])
        return F, ev, time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        res = list(ex.map(one, insts))
    wall = time.perf_counter() - t0
    F = np.array([r[0] for r in res], np.int64)
    out = {"what": "oracle VND (Algorithm 1) from the initial solution, one instance per host thread",
           "mean_F": float(F.mean()), "move_evals": int(sum(r[1] for r in res)),
           "cpu_s_per_instance": float(np.mean([r[2] for r in res])), "wall_s": wall, "threads": nthreads}
    if target_best is not None:
        out["best_on"] = int((F <= target_best).sum())
        out["mean_gap_pct"] = float(((F - target_best) / target_best).mean() * 100)
    return out


def workload_insts(name):
    from paper_1704_05132_amd.instances import WORKLOADS, workload
    w = WORKLOADS[name]
    return w, [workload(name, i) for i in range(w["n_inst"])]


def main():
    args = parse()
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU; a multi-GPU run is not supported (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_05132_amd import autotune, vns

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.valu_probe:
        print(json.dumps(valu_probe()), flush=True)
        return
    stream = torch.cuda.current_stream()
    table = autotune.TuneTable(TUNE_FILE)
    name = args.workload
    w, insts = workload_insts(name)
    key = autotune.signature(insts, w["chains"])
    iters = args.search_iters or w["iters"]
    t_start = time.perf_counter()

    # --- the workload's plain search over its iterations, in launches of --chunk; the timed sweeps run on the
    #     states it reached, and its per-instance bests are the learned search's targets ---
    if args.only_sweep:   # one search launch (a profiler sees one dispatch of the search kernel)
        plain = None
        warm_search(vns, lambda: new_ctx(vns, insts, w, stream, table, key))
        ctx = new_ctx(vns, insts, w, stream, table, key)
        search_main = search_once(vns, ctx, iters)
        search_main["best_F_sum"] = int(ctx.costs()[1].reshape(len(insts), w["chains"]).min(1).sum())
    else:
        plain = chunked_search(lambda: new_ctx(vns, insts, w, stream, table, key), len(insts), w["chains"], iters,
                               args.chunk, keep=True)
        ctx = plain.pop("ctx")
        search_main = {"iters": iters, "launches": len(plain["hist"]), "iters_per_launch": args.chunk,
                       "device_ms": plain["total_ms"], "move_evals": plain["evals"],
                       "value": plain["evals"] / (plain["total_ms"] / 1e3), "unit": "move-evals/s",
                       "best_F_sum": int(plain["best"].sum())}
    Ks = [i.K for i in insts]
    Ts = sorted({i.T for i in insts})
    sweep = sweep_steps(torch, vns, ctx, stream, args.steps, args.warmup)
    ctx.close()
    out_ttb = None
    if name in LEARNED_SETUP and not args.no_learned and not args.only_sweep:
        out_ttb = learned_vs_plain(args, vns, stream, table, key, name, insts, w, plain)

    config = {"workload": name, "instances": len(insts), "K": Ks[0] if len(Ks) == 1 else [min(Ks), max(Ks)],
              "T": Ts[0] if len(Ts) == 1 else Ts, "chains_per_instance": w["chains"],
              "chains": len(insts) * w["chains"], "neighbourhoods": ["flip_zM", "flip_zR", "shift"], "k_max": 5,
              "seed": w["seed"], "search_iters": iters, "tuning": (table.get(key) or {}).get("choice"),
              "step": "one exact sweep of every move of flip zM, flip zR and shift for every chain (k_eval), then "
                      "each chain's (price, slot) argmin (k_chain_best) copied to the host; on the states of "
                      f"the plain search after {iters} iterations"}
    out = {
        "metric": METRIC, "value": sweep["value"], "unit": "move-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sweep["device_ms"] / max(args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic", "config": config,
        "move_evals_per_step": sweep["move_evals_per_step"], "wall_s": sweep["wall_s"],
        "roofline": {"kernel": sweep["kernel"], "launch": SWEEP_LAUNCH, "bound": "alu", "achieved": sweep["achieved"],
                     "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s", "frac": sweep["frac"],
                     "traffic": measured_traffic(sweep["kernel"], name, "sweep"),
                     "kernel_ms_mean": sweep["kernel_ms_mean"], "ops_per_period_step": OPS_PER_PERIOD_STEP,
                     "accumulators": "int32 under the create-time bounds; costs int64"},
        "sweeps": {name: sweep},
        "search": {name: search_main},
    }
    if out_ttb is not None:
        out["time_to_plain_best"] = out_ttb

    if not args.only_sweep:
        # the other configurations' searches over their own iterations, and their sweeps
        for other in ("plain_100x52", "batched_4096"):
            if other == name:
                continue
            w2, insts2 = workload_insts(other)
            key2 = autotune.signature(insts2, w2["chains"])
            warm_search(vns, lambda: new_ctx(vns, insts2, w2, stream, table, key2))
            c2 = new_ctx(vns, insts2, w2, stream, table, key2)
            s2 = search_once(vns, c2, w2["iters"])
            out["search"][other] = s2
            out["sweeps"][other] = sweep_steps(torch, vns, c2, stream, max(args.steps, 20), args.warmup)
            c2.close()
            if other == "plain_100x52" and not args.no_learned:
                p2 = chunked_search(lambda: new_ctx(vns, insts2, w2, stream, table, key2), 1, w2["chains"],
                                    w2["iters"], args.chunk)
                out["time_to_plain_best_100x52"] = learned_vs_plain(args, vns, stream, table, key2, other, insts2,
                                                                    w2, p2)
    if not args.only_sweep and not args.no_quality:
        out["paper_quality"] = paper_quality(args, vns, stream)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    torch.cuda.synchronize()
    out["gpu_wall_s"] = time.perf_counter() - t_start
    if not args.no_cpu_baseline and not args.only_sweep:
        out["cpu_baseline"] = cpu_baseline(insts, w, name, args.cpu_seconds)
        if "paper_quality" in out:
            out["paper_quality"]["serial_vnd"] = serial_vnd_arm(getattr(paper_quality, "best_per_instance", None))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
