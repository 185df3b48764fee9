"""GPU: parity at the benchmarked sizes, in the launch configuration bench.py times (tuned launch shape,
one launch for all iterations).

The oracle re-prices every product in every VND pass (Algorithm 1 as written), so a whole 2000-iteration
chain takes it minutes. At full size the checks are therefore:
  * sampled chains: the first iterations' records equal the oracle's, record for record;
  * every sampled chain's final solution: its objective is exact and it is a local optimum of every
    neighbourhood (oracle prices of all its moves);
  * every chain: the records are consistent (acceptance iff strictly better, best non-increasing);
  * full sweeps at full size: every slot price of sampled chains equals the oracle's.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import WORKLOADS, workload

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_1704_05132_amd", "tune_table.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vns():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1704_05132_amd import vns as v
    return v


def tuned_context(vns, name, insts, options=None):
    from paper_1704_05132_amd import autotune
    w = WORKLOADS[name]
    ctx = vns.Context(insts if len(insts) > 1 else insts[0], seed=w["seed"], chains=w["chains"], nb_list=w["nb"],
                      options=options)
    table = autotune.TuneTable(TUNE)
    table.apply(ctx, autotune.signature(insts, w["chains"]))
    return ctx


def check_records(rec):
    """x only moves on strict improvement, so it is the best so far: accepted iff F_local < previous best."""
    acc = rec["accepted"] == 1
    assert (np.diff(rec["F_best"]) <= 0).all()
    assert (acc[1:] == (rec["F_local"][1:] < rec["F_best"][:-1])).all()
    assert (rec["F_local"] <= rec["F_shaken"]).all()


def check_final(ctx, g, inst):
    zM, zR = ctx.solution(g)
    F, Fb = ctx.cost(g)
    assert F == oracle.objective(inst, zM, zR)[0]
    price, _ = oracle.price_all(inst, zM, zR, 7)
    assert price.min() >= F   # no improving move in any neighbourhood


def check_prefix(ctx, g, inst, seed, n, nb=(1, 2, 4)):
    ref = oracle.Chain(inst, seed, g, nb).run(n)
    assert (ctx.trajectory(g)[:n] == ref).all(), g


def test_plain_100x52_bench_launch(vns):
    name = "plain_100x52"
    w = WORKLOADS[name]
    inst = workload(name)
    with tuned_context(vns, name, [inst]) as ctx:
        say(f"  {name}: {w['chains']} chains x {w['iters']} iterations, one launch")
        ctx.run(w["iters"])
        from paper_1704_05132_amd import autotune
        choice = autotune.TuneTable(TUNE).get(autotune.signature([inst], w["chains"]))["choice"]
        assert ctx.stats()["last_run_spec_iters"] == choice.get("iters", 1)   # the launch bench.py times
        for g in range(ctx.n_chains):
            rec = ctx.trajectory(g)
            assert len(rec) == w["iters"] and (rec["iter"] == np.arange(w["iters"])).all()
            check_records(rec)
        for g in (0, 37, 63):
            say(f"    chain {g}: first 100 records vs the oracle, final local optimum")
            check_prefix(ctx, g, inst, w["seed"], 100)
            check_final(ctx, g, inst)
        # full sweep of all 64 chains at this state: every slot of two chains against the oracle
        prices = ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=True)["slot_price"]
        for g in (5, 50):
            zM, zR = ctx.solution(g)
            ref, _ = oracle.price_all(inst, zM, zR, 7)
            got = prices[g * inst.K * 4 * inst.T:(g + 1) * inst.K * 4 * inst.T]
            assert (got == ref).all(), g


def test_batched_4096_bench_launch(vns):
    name = "batched_4096"
    w = WORKLOADS[name]
    insts = [workload(name, i) for i in range(w["n_inst"])]
    iters = 200
    with tuned_context(vns, name, insts, options={vns.OPT_TRACE: 1}) as ctx:
        say(f"  {name}: {len(insts)} instances x {w['chains']} chains x {iters} iterations, one launch")
        ctx.run(iters)
        rng = np.random.default_rng(7)
        for i in rng.choice(len(insts), 4, replace=False).tolist():
            g = i * w["chains"] + int(rng.integers(0, w["chains"]))
            say(f"    instance {i} (K={insts[i].K}, T={insts[i].T}) chain {g}")
            check_records(ctx.trajectory(g))
            check_prefix(ctx, g, insts[i], w["seed"], 30)
            check_final(ctx, g, insts[i])


def test_learned_batched_1024_launch(vns):
    name = "learned_batched_1024"
    w = WORKLOADS[name]
    insts = [workload(name, i) for i in range(w["n_inst"])]
    small = sorted(range(len(insts)), key=lambda i: insts[i].K * insts[i].T)[:3]
    with tuned_context(vns, name, insts) as ctx:
        say(f"  {name}: {len(insts)} instances x {w['chains']} chains, 3 iterations, one launch")
        ctx.run(3)
        for i in small:
            g = i * w["chains"] + 5
            say(f"    instance {i} (K={insts[i].K}, T={insts[i].T}) chain {g}")
            check_prefix(ctx, g, insts[i], w["seed"], 3)
            check_final(ctx, g, insts[i])
    # the learned search fused in the same persistent kernel: exact objectives and local optima
    with tuned_context(vns, name, insts, options={vns.OPT_LEARNED: 100}) as ctx:
        ctx.run(2)
        st = ctx.stats()
        assert st["last_run_learned_evals"] > 0
        for i in small:
            g = i * w["chains"] + 2
            check_records(ctx.trajectory(g))
            check_final(ctx, g, insts[i])
