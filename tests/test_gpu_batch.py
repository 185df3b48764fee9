"""GPU: batched persistent search, graph replay and launch-shape invariance, against the CPU oracle.

  * the 4096-instance workload (K ~ U{10..200}, T in {12, 24, 52}, 8 chains each) in one launch: sampled
    (instance, chain) trajectories bit-exact against the oracle;
  * a HIP-graph-captured search replayed several times, with other device work and synchronisations between
    replays, equals one eager run of all the iterations, and the oracle;
  * wavefronts per workgroup and the LDS budget change only time, never a record;
  * the autotuner's measured choice runs and leaves results unchanged.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vns():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1704_05132_amd import vns as v
    return v


@pytest.fixture(scope="module")
def batch():
    return [workload("batched_4096", i) for i in range(4096)]


def check_chain(ctx, g, inst, seed, iters, nb=(1, 2, 4)):
    ref = oracle.Chain(inst, seed, g, nb)
    rr = ref.run(iters)
    rg = ctx.trajectory(g)
    assert (rg == rr).all(), (g, inst.tag)
    zM, zR = ctx.solution(g)
    assert (zM == ref.zM).all() and (zR == ref.zR).all()
    assert ctx.cost(g) == (ref.F, ref.F_best)


def test_batched_4096_instances_one_launch(vns, batch):
    chains, iters = 8, 6
    say(f"  batch 4096 instances x {chains} chains x {iters} iterations")
    with vns.Context(batch, seed=3, chains=chains) as ctx:
        assert ctx.n_chains == 4096 * chains
        ctx.run(iters)
        st = ctx.stats()
        assert st["last_run_evals"] > 0
        rng = np.random.default_rng(41)
        picks = set(rng.choice(4096, size=10, replace=False).tolist())
        picks.add(int(np.argmax([i.K for i in batch])))
        for i in sorted(picks):
            c = int(rng.integers(0, chains))
            say(f"    instance {i} K={batch[i].K} T={batch[i].T} chain {c}")
            check_chain(ctx, i * chains + c, batch[i], 3, iters)


def test_graph_replay_equals_eager_run(vns):
    insts = [workload("batched_4096", i) for i in range(6)]
    chains = 3
    say("  graph replay x3 vs eager")
    with vns.Context(insts, seed=3, chains=chains, options={vns.OPT_GRAPH: 1}) as gctx, \
            vns.Context(insts, seed=3, chains=chains) as ectx:
        parts = []
        for rep in range(3):
            gctx.run(7)
            parts.append([gctx.trajectory(g) for g in range(gctx.n_chains)])
            # other device work and host synchronisation between replays
            gctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False)
            gctx.cost(0)
        ectx.run(21)
        for g in range(ectx.n_chains):
            rg = np.concatenate([p[g] for p in parts])
            re = ectx.trajectory(g)
            assert (rg == re).all(), g
            assert (rg["iter"] == np.arange(21)).all()
            sa, sb = gctx.solution(g), ectx.solution(g)
            assert (sa[0] == sb[0]).all() and (sa[1] == sb[1]).all()
        for g in (0, 4, 17):
            check_chain(ectx, g, insts[g // chains], 3, 21)


@pytest.mark.parametrize("waves,lds", [(1, 0), (2, 65536), (4, 0), (8, 65536), (3, 4096)])
def test_launch_shape_does_not_change_results(vns, waves, lds):
    insts = [workload("batched_4096", i) for i in range(8)]
    say(f"  shape waves={waves} lds={lds}")
    with vns.Context(insts, seed=3, chains=2) as ref_ctx, \
            vns.Context(insts, seed=3, chains=2, options={vns.OPT_RUN_WAVES: waves, vns.OPT_RUN_LDS: lds}) as ctx:
        ref_ctx.run(12)
        ctx.run(12)
        for g in range(ctx.n_chains):
            assert (ctx.trajectory(g) == ref_ctx.trajectory(g)).all(), g


def test_autotuner_choice_runs_and_keeps_results(vns, tmp_path):
    from paper_1704_05132_amd import autotune
    insts = [workload("batched_4096", i) for i in range(32)]
    say("  autotune 32 instances")
    best, timings = autotune.tune_search(insts, seed=3, chains=2, iters=4,
                                         candidates=[dict(waves=2, lds=0), dict(waves=4, lds=65536)])
    assert best in [c for c, _ in timings] and all(ms > 0 for _, ms in timings)
    table = autotune.TuneTable(tmp_path / "tune.json")
    key = autotune.signature(insts, 2)
    table.put(key, best, timings)
    with vns.Context(insts, seed=3, chains=2) as ctx, vns.Context(insts, seed=3, chains=2) as plain:
        assert table.apply(ctx, key)
        best_e, _ = autotune.tune_eval(ctx, reps=2, candidates=[dict(group=1), dict(group=2)])
        ctx.run(5)
        plain.run(5)
        for g in range(ctx.n_chains):
            assert (ctx.trajectory(g) == plain.trajectory(g)).all()


@pytest.mark.parametrize("nb", [(1, 2, 4), (4, 2, 1), (1, 2), (2,)])
def test_speculative_vnd_equals_sequential(vns, nb):
    """Grouped speculative VND against one wavefront per product: same records, same solutions and the same
    number of consumed move-evaluations (discarded speculative pricing is not counted)."""
    insts = [workload("batched_4096", i) for i in range(3)] + [workload("plain_100x52")]
    say(f"  speculative vs sequential nb={nb}")
    with vns.Context(insts, seed=3, chains=4, nb_list=nb, options={vns.OPT_SPECULATE: 1}) as sp, \
            vns.Context(insts, seed=3, chains=4, nb_list=nb, options={vns.OPT_SPECULATE: 0}) as sq:
        for rep in range(2):
            sp.run(15)
            sq.run(15)
            assert sp.stats()["last_run_evals"] == sq.stats()["last_run_evals"]
            for g in range(sp.n_chains):
                assert (sp.trajectory(g) == sq.trajectory(g)).all(), g
        for g in range(sp.n_chains):
            a, b = sp.solution(g), sq.solution(g)
            assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


@pytest.mark.parametrize("learned", [0, 100])
def test_state_in_lds_does_not_change_results(vns, learned):
    """The chains' solution state kept in LDS for the launch, or in device memory: same records, solutions
    and costs, for the plain and the learned search."""
    insts = [workload("batched_4096", i) for i in range(5)] + [workload("plain_100x52")]
    say(f"  state in LDS vs device memory, learned={learned}")
    opts = {vns.OPT_LEARNED: learned} if learned else {}
    with vns.Context(insts, seed=3, chains=3, options={**opts, vns.OPT_STATE_LDS: 1}) as a, \
            vns.Context(insts, seed=3, chains=3, options={**opts, vns.OPT_STATE_LDS: 0}) as b:
        for rep in range(2):
            a.run(9)
            b.run(9)
            for g in range(a.n_chains):
                assert (a.trajectory(g) == b.trajectory(g)).all(), g
        assert (a.costs()[0] == b.costs()[0]).all() and (a.costs()[1] == b.costs()[1]).all()
        for g in range(a.n_chains):
            sa, sb = a.solution(g), b.solution(g)
            assert (sa[0] == sb[0]).all() and (sa[1] == sb[1]).all()


@pytest.mark.parametrize("learned", [0, 100])
def test_vnd_memo_keeps_the_trajectory(vns, learned):
    """Skipping neighbourhoods already priced without improvement on the same pattern applies the same
    moves: identical records and solutions (and the oracle's, for the plain search), fewer evaluations."""
    insts = [workload("batched_4096", i) for i in range(4)] + [workload("plain_100x52")]
    say(f"  VND memo on vs off, learned={learned}")
    opts = {vns.OPT_LEARNED: learned} if learned else {}
    with vns.Context(insts, seed=3, chains=3, options={**opts, vns.OPT_VND_MEMO: 1}) as a, \
            vns.Context(insts, seed=3, chains=3, options={**opts, vns.OPT_VND_MEMO: 0}) as b:
        a.run(25)
        b.run(25)
        ea, eb = a.stats()["last_run_evals"], b.stats()["last_run_evals"]
        say(f"    evaluations {ea} with the skip, {eb} without")
        assert ea < eb
        for g in range(a.n_chains):
            assert (a.trajectory(g) == b.trajectory(g)).all(), g
            sa, sb = a.solution(g), b.solution(g)
            assert (sa[0] == sb[0]).all() and (sa[1] == sb[1]).all()
        if not learned:
            for g in (0, 7, 14):
                check_chain(a, g, insts[g // 3], 3, 25)
