"""Autotuner for the launch shape of the search and pricing kernels.

The search kernel runs one workgroup per chain; how many wavefronts a workgroup has (so how many of a
chain's products run their VND side by side), whether the neighbourhoods of one product's VND are priced
side by side by a group of wavefronts (speculative VND, `spec`) and how much LDS it may use to keep an
instance's rows resident trade occupancy against parallelism, and the best choice depends on K, T and the
number of chains.  The pricing kernel's tuning knob is how many chains of an instance share one workgroup, or the
range form with its wavefronts per workgroup (`spread`: the pairs split evenly over the compute units).  Results
never depend on these choices (the kernels compute the same exact costs and trajectories); only time does.

`tune_search` and `tune_eval` time each candidate on the actual workload with the library's own device
timers and return the fastest; `TuneTable` persists choices per workload signature in JSON.
"""
from __future__ import annotations

import json
from pathlib import Path
from typing import Callable, Iterable, Sequence

SEARCH_CANDIDATES = ([dict(waves=w, lds=l, spec=0, state=st) for w in (2, 4, 8) for l in (0, 65536) for st in (0, 1)] +
                     [dict(spec=1, spec_waves=s, lds=l) for s in (6, 9, 15) for l in (0, 65536)] +
                     [dict(waves=w, lds=65536, spec=0, iters=m) for w, m in
                      ((8, 2), (8, 3), (8, 4), (4, 3), (4, 4), (4, 6), (4, 8), (4, 12), (3, 8), (3, 12), (2, 6),
                       (2, 8))])
EVAL_CANDIDATES = [dict(group=g) for g in (1, 2, 3, 4, 5, 6, 8, 12, 16)] + [dict(spread=w) for w in (4, 8, 12, 16)]


def signature(instances, chains: int) -> str:
    """Workload key: instance count, K range, the set of horizons, chains per instance."""
    Ks = [i.K for i in instances]
    Ts = sorted({i.T for i in instances})
    return f"n{len(instances)}_K{min(Ks)}-{max(Ks)}_T{'-'.join(map(str, Ts))}_c{chains}"


def pick(candidates: Iterable[dict], measure: Callable[[dict], float]):
    """Measure every candidate; return (fastest, [(candidate, ms), ...]).  Ties keep the earlier one."""
    timings = []
    best, best_ms = None, None
    for cand in candidates:
        ms = float(measure(cand))
        timings.append((dict(cand), ms))
        if best_ms is None or ms < best_ms:
            best, best_ms = dict(cand), ms
    return best, timings


def tune_search(instances, seed: int, chains: int, nb_list: Sequence[int] = (1, 2, 4), iters: int = 20,
                candidates: Sequence[dict] = tuple(SEARCH_CANDIDATES), warmup: int = 0):
    """Time `iters` GVNS iterations (one launch) after `warmup` untimed ones, on a fresh context, for each
    launch-shape candidate.  The first iterations run the VND of every product; later ones only of the
    shaken products, so a warm-up tunes for the steady state.  A speculative-iterations candidate whose run
    fell back to one workgroup per chain (its workgroups do not all fit at once) is timed as infinite: it
    is another candidate under a different name."""
    from . import vns

    def measure(c):
        with vns.Context(instances, seed=seed, chains=chains, nb_list=nb_list, trace=False,
                         options=search_options(c)) as ctx:
            if warmup > 0:
                ctx.run(warmup)
            ctx.run(iters)
            st = ctx.stats()
            if st["last_run_spec_iters"] != c.get("iters", 1):
                return float("inf")
            return st["last_run_ms"]

    return pick(candidates, measure)


def search_options(c: dict) -> dict:
    """Context options of a search candidate (keys waves, lds, spec, spec_waves, state, iters = speculative
    iterations per chain; missing keys keep defaults)."""
    from . import vns
    opts = {}
    if "waves" in c:
        opts[vns.OPT_RUN_WAVES] = c["waves"]
    if "lds" in c:
        opts[vns.OPT_RUN_LDS] = c["lds"]
    if "spec" in c:
        opts[vns.OPT_SPECULATE] = c["spec"]
    if "spec_waves" in c:
        opts[vns.OPT_SPEC_WAVES] = c["spec_waves"]
    if "state" in c:
        opts[vns.OPT_STATE_LDS] = c["state"]
    if "iters" in c:
        opts[vns.OPT_SPEC_ITERS] = c["iters"]
    return opts


def eval_options(c: dict) -> dict:
    """Pricing-kernel options of a tuning choice: the range form (`spread`) or chains per workgroup (`group`)."""
    from . import vns
    opts = {vns.OPT_EVAL_SPREAD: int(c.get("spread", 0))}
    if "group" in c:
        opts[vns.OPT_EVAL_GROUP] = c["group"]
    return opts


def tune_eval(ctx, nb_mask: int = 7, reps: int = 5, candidates: Sequence[dict] = tuple(EVAL_CANDIDATES)):
    """Median device time of a full pricing sweep of every chain of ctx for each pricing launch shape."""
    from . import vns

    def measure(c):
        for opt, v in eval_options(c).items():
            ctx.set_option(opt, v)
        ms = []
        for _ in range(reps):
            ctx.eval_neighbourhood(nb_mask, vns.ALL_CHAINS, slot_prices=False)
            ms.append(ctx.stats()["last_eval_ms"])
        return sorted(ms)[len(ms) // 2]

    best, timings = pick(candidates, measure)
    for opt, v in eval_options(best).items():
        ctx.set_option(opt, v)
    return best, timings


class TuneTable:
    """Choices per workload signature, stored as JSON."""

    def __init__(self, path):
        self.path = Path(path)
        self.data = json.loads(self.path.read_text()) if self.path.exists() else {}

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, choice: dict, timings=None):
        self.data[key] = {"choice": choice, "timings_ms": [[c, ms] for c, ms in (timings or [])]}
        self.path.write_text(json.dumps(self.data, indent=1, sort_keys=True))

    def apply(self, ctx, key: str) -> bool:
        """Set the stored search/eval options on ctx; False if the table has no entry for key."""
        from . import vns
        e = self.get(key)
        if not e:
            return False
        ch = e["choice"]
        for opt, v in search_options(ch).items():
            ctx.set_option(opt, v)
        for opt, v in eval_options(ch).items():
            ctx.set_option(opt, v)
        return True
