#!/usr/bin/env python3
"""Benchmark of the MI355X lot-sizing VNS: exact move-evaluations per second.

Workload: one synthetic instance of 100 products x 52 periods (demand U{0..200}, returns floor(D*U(0.2,0.8)),
setup costs U{200..2000}, holding hM U{2..6}, hR U{1..hM}; seed 2), 64 independent Philox chains, neighbourhoods
flip zM, flip zR, shift; shake sizes 1..5.  One step = one GVNS iteration (shake, VND, acceptance) of all 64
chains; the K timed steps are one vns_run(K) launch on a fresh context starting from the initial solution,
so the timed region is exactly the workload's first K iterations.  Inputs are resident in HBM before timing.

Prints one JSON line.  Extra fields: the full-neighbourhood sweep of all chains (the pricing kernel alone),
the dominant kernel's roofline, and the CPU oracle timed on this host on a bounded sample.  --workload
batched_4096 runs the 4096-instance batch (K ~ U{10..200}, T in {12, 24, 52}, 8 chains each) in one launch
instead.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one int32 op per lane per clock)
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
OPS_PER_PERIOD_STEP = 14     # operations of one period-step of the forward decode
TUNE_FILE = os.path.join(ROOT, "paper_1704_05132_amd", "tune_table.json")


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


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it is current."""
    try:
        with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="plain_100x52", choices=["plain_100x52", "plain_10x12", "batched_4096"])
    ap.add_argument("--graph", action="store_true", help="run the search through a captured HIP graph")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration for profiling runs)")
    return ap.parse_args()


def cpu_baseline(pairs, nb, target_s, label):
    """The oracle, as it is, on this host: independent (instance, seed, chain) runs from iteration 0, one per
    thread, each sized so that the sample takes about target_s."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1, len(pairs)))
    pairs = pairs[:threads]
    inst, seed, chain = pairs[0]
    probe = oracle.Chain(inst, seed, chain, nb)
    t0 = time.perf_counter()
    probe.run(4)
    per_first4 = time.perf_counter() - t0
    t0 = time.perf_counter()
    probe.run(8)
    per_iter = (time.perf_counter() - t0) / 8
    iters = int(max(5, 4 + (target_s - per_first4) / max(per_iter, 1e-6)))

    def one(p):
        ch = oracle.Chain(p[0], p[1], p[2], nb)
        ch.run(iters)
        return ch.evals

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        evals = sum(ex.map(one, pairs))
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "move-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} chains x {iters} GVNS iterations of {label} from iteration 0, one chain per "
                      f"thread ({evals} move-evaluations in {dt:.1f} s)"}


def main():
    args = parse()
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; a multi-GPU run is not part of it (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_05132_amd import autotune, vns
    from paper_1704_05132_amd.instances import WORKLOADS, workload

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    name = args.workload
    w = WORKLOADS[name]
    insts = [workload(name, i) for i in range(w["n_inst"])]
    target = insts[0] if len(insts) == 1 else insts
    chains = w["chains"]
    stream = torch.cuda.current_stream()
    table = autotune.TuneTable(TUNE_FILE)
    key = autotune.signature(insts, chains)

    def make(trace):
        c = vns.Context(target, seed=w["seed"], chains=chains, nb_list=w["nb"], trace=trace,
                        options={vns.OPT_GRAPH: 1} if args.graph else None)
        c.bind_stream(stream)
        table.apply(c, key)
        return c

    # --- warmup: W iterations on a separate context (same data), then sweeps ---
    warm = make(False)
    if args.warmup > 0:
        warm.run(args.warmup)
    warm.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False)

    # --- timed: K iterations of all chains in one launch, from the initial solution ---
    ctx = make(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    st = ctx.stats()
    run_ms = st["last_run_ms"]          # HIP events around the search launch on the context stream
    evals = st["last_run_evals"]
    value = evals / (ev_ms / 1e3)
    ms_per_step = ev_ms / args.steps

    # best cost of the plain method per instance (over its chains) and the iteration it was first reached
    bests = []
    for i in range(len(insts)):
        bF, bit = None, None
        for c in range(chains):
            rec = ctx.trajectory(i * chains + c)
            fb = int(rec["F_best"][-1])
            it = int(rec["iter"][int((rec["F_best"] == fb).argmax())])
            if bF is None or fb < bF or (fb == bF and it < bit):
                bF, bit = fb, it
        bests.append((bF, bit))
    last_it = max(it for _, it in bests)

    # --- full-neighbourhood sweep of all chains (pricing kernel alone) ---
    sweep_ms, sweep_ev, sweep_steps = [], 0, 0
    for _ in range(args.sweep_reps):
        ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False)
        s = ctx.stats()
        sweep_ms.append(s["last_eval_ms"])
        sweep_ev, sweep_steps = s["last_eval_evals"], s["last_eval_period_steps"]
    sweep_med = statistics.median(sweep_ms)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    peak = VALU_PEAK_OPS / 1e12
    achieved = st["last_run_period_steps"] * OPS_PER_PERIOD_STEP / (run_ms / 1e3) / 1e12
    sweep_achieved = sweep_steps * OPS_PER_PERIOD_STEP / (sweep_med / 1e3) / 1e12
    Ks = [i.K for i in insts]
    Ts = sorted({i.T for i in insts})
    config = {"workload": name, "instances": len(insts), "K": Ks[0] if len(Ks) == 1 else [min(Ks), max(Ks)],
              "T": Ts[0] if len(Ts) == 1 else Ts, "chains": chains, "iters": args.steps,
              "neighbourhoods": ["flip_zM", "flip_zR", "shift"], "k_max": 5, "seed": w["seed"],
              "graph": bool(args.graph), "tuning": (table.get(key) or {}).get("choice"),
              "step": "one GVNS iteration of all chains; K steps = one vns_run(K) launch"}
    out = {
        "metric": "exact move-evals/s (int64 cost) + time-to-plain-best-cost, learned vs plain",
        "value": value,
        "unit": "move-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
        "result_dtype": "int64",
        "move_evals": evals,
        "wall_s": wall,
        "kernel_ms": run_ms,
        "plain_best": ({"F": bests[0][0], "iteration": bests[0][1], "ms": (bests[0][1] + 1) * ms_per_step}
                       if len(insts) == 1 else
                       {"F_sum": int(sum(f for f, _ in bests)), "last_iteration_improved": last_it,
                        "ms": (last_it + 1) * ms_per_step}),
        "roofline": {"kernel": "k_run", "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic("k_run", name),
                     "ops_per_period_step": OPS_PER_PERIOD_STEP},
        "sweep": {"kernel": "k_eval", "move_evals": sweep_ev, "median_ms": sweep_med,
                  "value": sweep_ev / (sweep_med / 1e3), "unit": "move-evals/s", "achieved": sweep_achieved,
                  "peak": peak, "frac": sweep_achieved / peak, "traffic": measured_traffic("k_eval", name)},
    }
    if not args.no_cpu_baseline:
        rng = __import__("numpy").random.default_rng(0)
        order = rng.permutation(len(insts)) if len(insts) > 1 else [0] * 16
        pairs = [(insts[i], w["seed"], int(i) * chains + (j % chains)) for j, i in enumerate(list(order)[:16])]
        out["cpu_baseline"] = cpu_baseline(pairs, w["nb"], args.cpu_seconds, name)
    print(json.dumps(out), flush=True)
    ctx.close()
    warm.close()


if __name__ == "__main__":
    main()
