"""GPU: the best-of-G search (Algorithm 2: G shakes of the same solution, each followed by the VND, the
minimum kept), against the oracle's best-of-G chain.

  * G = 2, 4, 8 in the GVNS form (move iff strictly better, k schedule) and as printed (k fixed, the minimum
    always kept), record for record, with the final solutions and costs;
  * a run continued over several vns_run calls equals one run;
  * the selected stream is reported, and every stream is used;
  * combinations the search does not support, and too many workgroups to be resident, are errors.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import edge_instance, workload

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


def check(ctx, g, inst, seed, G, literal, iters, chain=None, k_max=5, nb=(1, 2, 4)):
    ref = oracle.BestOfChain(inst, seed, g if chain is None else chain, nb, k_max, G=G, literal=literal)
    rr = ref.run(iters)
    rg = ctx.trajectory(g)
    assert (rg == rr).all(), (g, inst.tag)
    zM, zR = ctx.solution(g)
    assert (zM == ref.zM).all() and (zR == ref.zR).all()
    assert ctx.cost(g) == (ref.F, ref.F_best)
    return rr


@pytest.mark.parametrize("G,literal", [(2, 0), (4, 0), (8, 0), (3, 1), (1, 1)])
def test_best_of_g_equals_oracle(vns, G, literal):
    inst = edge_instance("uniform", 12, 20, seed=5)
    chains, iters = 4, 30
    say(f"  best-of-{G} literal={literal}: {chains} chains x {iters} iterations")
    with vns.Context(inst, seed=6, chains=chains, options={vns.OPT_BEST_OF: G, vns.OPT_BEST_OF_LITERAL: literal,
                                                           vns.OPT_RUN_WAVES: 4}) as ctx:
        ctx.run(iters)
        winners = set()
        for g in range(chains):
            rr = check(ctx, g, inst, 6, G, bool(literal), iters)
            winners |= set(rr["winner"].tolist())
        if G > 2:
            assert len(winners) > 1   # more than one stream wins somewhere


def test_best_of_g_continues_across_runs(vns):
    inst = workload("plain_100x52")
    G, chains = 4, 8
    say(f"  best-of-{G}, 100x52 x {chains} chains: 5 + 12 + 8 iterations against one oracle run")
    with vns.Context(inst, seed=2, chains=chains, options={vns.OPT_BEST_OF: G}) as ctx:
        parts = []
        for n in (5, 12, 8):
            ctx.run(n)
            parts.append([ctx.trajectory(g) for g in range(chains)])
        for g in (0, 5):
            ref = oracle.BestOfChain(inst, 2, g, (1, 2, 4), 5, G=G)
            rr = ref.run(25)
            got = np.concatenate([p[g] for p in parts])
            assert (got == rr).all(), g
            zM, zR = ctx.solution(g)
            assert (zM == ref.zM).all() and (zR == ref.zR).all()


def test_best_of_g_batched_instances(vns):
    insts = [workload("batched_4096", i) for i in range(6)]
    G, chains, iters = 3, 2, 15
    say(f"  best-of-{G}, 6 batched instances x {chains} chains")
    with vns.Context(insts, seed=3, chains=chains, options={vns.OPT_BEST_OF: G, vns.OPT_RUN_WAVES: 2}) as ctx:
        ctx.run(iters)
        for i in (0, 4):
            for c in range(chains):
                g = i * chains + c
                check(ctx, g, insts[i], 3, G, False, iters, chain=g)


@pytest.mark.parametrize("case", ["learned", "log", "graph", "spec_iters", "too_many"])
def test_best_of_g_unsupported_is_an_error(vns, case):
    insts = [workload("batched_4096", i) for i in range(4)]
    chains, opts = 2, {vns.OPT_BEST_OF: 4}
    if case == "learned":
        opts[vns.OPT_LEARNED] = 100
    elif case == "log":
        opts[vns.OPT_LOG] = 4096
    elif case == "graph":
        opts[vns.OPT_GRAPH] = 1
    elif case == "spec_iters":
        opts[vns.OPT_SPEC_ITERS] = 4
    else:
        insts, chains = [workload("batched_4096", i) for i in range(512)], 8
    say(f"  best-of-G refuses: {case}")
    with vns.Context(insts, seed=5, chains=chains, options=opts) as ctx:
        with pytest.raises(vns.VNSError):
            ctx.run(3)


def test_best_of_option_range(vns):
    with vns.Context(workload("plain_10x12"), seed=1) as ctx:
        assert ctx.get_option(vns.OPT_BEST_OF) == 0 and ctx.get_option(vns.OPT_BEST_OF_LITERAL) == 0
        for bad in (-1, 17):
            with pytest.raises(vns.VNSError):
                ctx.set_option(vns.OPT_BEST_OF, bad)
        with pytest.raises(vns.VNSError):
            ctx.set_option(vns.OPT_BEST_OF_LITERAL, 2)
