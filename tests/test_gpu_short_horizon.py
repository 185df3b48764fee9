"""GPU: the short-horizon search kernel (k_run_short, launched when a batch has an instance with T <= 31)
against the oracle.

There the VND prices consecutive neighbourhoods of a pass side by side in one wavefront pass when their moves
fit 64 lanes (at most one swap list per pass), takes the first improving one in Algorithm 1's order and drops
the rest.  Records, solutions and costs must equal the oracle's one-at-a-time VND, and the counted
move-evaluations those of the same kernel with the move log on (which prices one neighbourhood at a time; the
device runs the VND of the shaken products only, so its counts are not the oracle's), for neighbourhood lists of
every order, repeated neighbourhoods (two shift neighbourhoods in a row),
single-neighbourhood lists, T = 1 .. 31 and the first horizon past it (32), degenerate instances, a batch
that mixes short and long horizons, the decode readings and shakes of every size.
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


def evals_one_at_a_time(vns, insts, chains, seed, iters, nb, kmax=5):
    """The same search with the move log on: the kernel then prices one neighbourhood per pass."""
    with vns.Context(insts if len(insts) > 1 else insts[0], seed=seed, chains=chains, k_max=kmax, nb_list=nb,
                     options={vns.OPT_LOG: 1 << 16}) as ctx:
        ctx.run(iters)
        return ctx.stats()["last_run_evals"]


def check(vns, ctx, insts, chains, seed, iters, nb, kmax=5):
    for g in range(ctx.n_chains):
        inst = insts[g // chains]
        ref = oracle.Chain(inst, seed, g, nb, kmax)
        rr = ref.run(iters)
        rg = ctx.trajectory(g)
        bad = np.flatnonzero(rg != rr)
        assert len(bad) == 0, (g, inst.K, inst.T, bad[:5])
        zM, zR = ctx.solution(g)
        assert (zM == ref.zM).all() and (zR == ref.zR).all(), g
        assert ctx.cost(g) == (ref.F, ref.F_best), g
    assert ctx.stats()["last_run_evals"] == evals_one_at_a_time(vns, insts, chains, seed, iters, nb, kmax)


NB_LISTS = [(1, 2, 4), (4, 1, 2), (2, 4, 1), (4, 4, 1, 2), (1, 1, 2), (4,), (2, 4, 4, 1), (1, 4)]


@pytest.mark.parametrize("nb", NB_LISTS)
@pytest.mark.parametrize("kind,K,T", [("uniform", 6, 12), ("big_returns", 5, 24), ("sparse", 4, 31)])
def test_neighbourhood_lists(vns, nb, kind, K, T):
    inst = edge_instance(kind, K, T, seed=K + T)
    iters, seed = 30, 13
    say(f"  short horizon {kind} {K}x{T} nb={nb}")
    with vns.Context(inst, seed=seed, chains=3, nb_list=nb) as ctx:
        ctx.run(iters)
        check(vns, ctx, [inst], 3, seed, iters, nb)


@pytest.mark.parametrize("kind,K,T,kmax", [("uniform", 3, 1, 5), ("uniform", 4, 2, 5), ("zero_demand", 3, 5, 5),
                                           ("no_returns", 5, 9, 3), ("returns_eq_demand", 4, 16, 7),
                                           ("zero_costs", 3, 20, 5), ("uniform", 8, 31, 64), ("uniform", 5, 32, 5)])
def test_edge_instances(vns, kind, K, T, kmax):
    inst = edge_instance(kind, K, T, seed=3)
    iters, seed = 40, 7
    with vns.Context(inst, seed=seed, chains=2, k_max=kmax) as ctx:
        ctx.run(iters)
        check(vns, ctx, [inst], 2, seed, iters, (1, 2, 4), kmax)


def test_mixed_batch_over_several_runs(vns):
    insts = [edge_instance("uniform", 7, 12, seed=1), workload("batched_4096", 5), edge_instance("sparse", 3, 52, seed=2),
             edge_instance("big_returns", 6, 24, seed=3), edge_instance("uniform", 2, 104, seed=4)]
    chains, seed = 2, 21
    say("  short horizon: mixed batch " + " ".join(f"{i.K}x{i.T}" for i in insts))
    with vns.Context(insts, seed=seed, chains=chains) as ctx:
        ctx.run(9)
        ctx.run(11)
        for g in range(ctx.n_chains):
            inst = insts[g // chains]
            ref = oracle.Chain(inst, seed, g)
            ref.run(9)
            rr = ref.run(11)
            assert (ctx.trajectory(g) == rr).all(), g
            zM, zR = ctx.solution(g)
            assert (zM == ref.zM).all() and (zR == ref.zR).all(), g


@pytest.mark.parametrize("model", [1, 2, 3])
def test_decode_readings(vns, model):
    inst = edge_instance("big_returns", 6, 20, seed=model)
    inst.strict = bool(model & 1)
    inst.dispose = bool(model & 2)
    iters, seed = 30, 5
    with vns.Context(inst, seed=seed, chains=3) as ctx:
        assert ctx.get_option(vns.OPT_DECODE) == model
        ctx.run(iters)
        check(vns, ctx, [inst], 3, seed, iters, (1, 2, 4))
