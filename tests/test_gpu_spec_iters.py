"""GPU: speculative GVNS iterations (m workgroups per chain, one iteration each, resolved in order).

A rejected iteration leaves x unchanged, so iterations i+1..i+m-1 can be computed beside iteration i as if
it were rejected; what follows the first accepted one is thrown away (Section 3, the shake-VND-move-or-not
loop).  The search must not notice: every record, solution and counted move-evaluation equals the
one-workgroup search's, and sampled chains equal the oracle; for the learned search the neighbourhood and
fallback counts too.  A run that cannot use the cooperative launch (move log, graph capture, too many
workgroups to be resident) falls back to one workgroup per chain and says so in its statistics.
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


def same_search(a, b, n_chains):
    for g in range(n_chains):
        assert (a.trajectory(g) == b.trajectory(g)).all(), g
        za, ra = a.solution(g)
        zb, rb = b.solution(g)
        assert (za == zb).all() and (ra == rb).all(), g
    (Fa, Fba), (Fb, Fbb) = a.costs(), b.costs()
    assert (Fa == Fb).all() and (Fba == Fbb).all()
    assert a.stats()["last_run_evals"] == b.stats()["last_run_evals"]


# 8 instances x 4 chains = 32 chains (the XCD-aware placement) and 1 instance x 3 chains (the plain one)
@pytest.mark.parametrize("m", [2, 4, 8, 16])
@pytest.mark.parametrize("layout", ["xcd", "plain"])
def test_speculative_iterations_equal_one_workgroup(vns, m, layout):
    if layout == "xcd":
        insts, chains = [workload("batched_4096", i) for i in range(8)], 4
    else:
        insts, chains = [workload("batched_4096", 5)], 3
    say(f"  spec_iters m={m} layout={layout}")
    # 16 iterations side by side: 4 wavefronts per workgroup, so that the 512 workgroups are resident at once
    opts = {vns.OPT_SPEC_ITERS: m, **({vns.OPT_RUN_WAVES: 4} if m > 8 else {})}
    with vns.Context(insts, seed=7, chains=chains) as ref, \
            vns.Context(insts, seed=7, chains=chains, options=opts) as ctx:
        for iters in (1, 40, 97):   # a chain's first iteration (a full sweep), then runs that continue it
            ref.run(iters)
            ctx.run(iters)
            st, rst = ctx.stats(), ref.stats()
            assert st["last_run_spec_iters"] == m and rst["last_run_spec_iters"] == 1
            assert rst["last_run_discarded_evals"] == 0
            # the first iteration of a chain runs alone; later rounds throw away what follows an acceptance
            assert (st["last_run_discarded_evals"] > 0) == (iters > 1)
            same_search(ctx, ref, ctx.n_chains)
        acc = sum(int(ctx.trajectory(g)["accepted"].sum()) for g in range(ctx.n_chains))
        assert 0 < acc < 97 * ctx.n_chains   # both outcomes occur, so rounds end early and run to the end


def test_speculative_iterations_equal_oracle(vns):
    inst = workload("plain_100x52")
    chains, iters, m = 8, 60, 4
    say(f"  spec_iters m={m} 100x52 x {chains} chains vs oracle, {iters} iterations")
    with vns.Context(inst, seed=11, chains=chains, options={vns.OPT_SPEC_ITERS: m}) as ctx:
        ctx.run(iters)
        assert ctx.stats()["last_run_spec_iters"] == m
        for g in (0, 5):
            ref = oracle.Chain(inst, 11, g, (1, 2, 4))
            rr = ref.run(iters)
            assert (ctx.trajectory(g) == rr).all(), g
            zM, zR = ctx.solution(g)
            assert (zM == ref.zM).all() and (zR == ref.zR).all()
            assert ctx.cost(g) == (ref.F, ref.F_best)


def test_speculative_iterations_headline_shape(vns):
    """The 100x52 instance with 64 chains, 8 wavefronts per workgroup and 4 iterations side by side: 256
    workgroups, one per compute unit."""
    inst = workload("plain_100x52")
    say("  spec_iters m=4 100x52 x 64 chains, waves 8, 150 iterations")
    opts = {vns.OPT_RUN_WAVES: 8, vns.OPT_RUN_LDS: 65536}
    with vns.Context(inst, seed=1, chains=64, options=opts) as ref, \
            vns.Context(inst, seed=1, chains=64, options={**opts, vns.OPT_SPEC_ITERS: 4}) as ctx:
        ref.run(150)
        ctx.run(150)
        assert ctx.stats()["last_run_spec_iters"] == 4
        same_search(ctx, ref, 64)


@pytest.mark.parametrize("case", ["log", "graph", "too_many"])
def test_speculative_iterations_fall_back(vns, case):
    insts = [workload("batched_4096", i) for i in range(4)]
    chains, opts = 2, {vns.OPT_SPEC_ITERS: 4}
    if case == "log":
        opts[vns.OPT_LOG] = 4096
    elif case == "graph":
        opts[vns.OPT_GRAPH] = 1
    else:   # more workgroups than the device holds at once
        insts, chains = [workload("batched_4096", i) for i in range(1024)], 8
    say(f"  spec_iters fallback: {case}")
    base = {k: v for k, v in opts.items() if k != vns.OPT_SPEC_ITERS}
    with vns.Context(insts, seed=5, chains=chains, options=base) as ref, \
            vns.Context(insts, seed=5, chains=chains, options=opts) as ctx:
        ref.run(6)
        ctx.run(6)
        assert ctx.stats()["last_run_spec_iters"] == 1
        for g in range(0, ctx.n_chains, max(1, ctx.n_chains // 16)):
            assert (ctx.trajectory(g) == ref.trajectory(g)).all(), g


def test_spec_iters_option_range(vns):
    with vns.Context(workload("plain_10x12"), seed=1) as ctx:
        assert ctx.get_option(vns.OPT_SPEC_ITERS) == 1
        for bad in (0, 17, -1):
            with pytest.raises(vns.VNSError):
                ctx.set_option(vns.OPT_SPEC_ITERS, bad)
        ctx.set_option(vns.OPT_SPEC_ITERS, 16)
        assert ctx.get_option(vns.OPT_SPEC_ITERS) == 16


# Degenerate instances: with zero costs or zero demand nothing ever improves, no iteration is accepted and
# x never becomes a local optimum, so every round shares one iteration over the chain's workgroups; a single
# product, k_max = 1 and horizons of 1 and 128 periods cover the other ends.
@pytest.mark.parametrize("kind,K,T,kmax", [
    ("zero_costs", 7, 12, 5), ("zero_demand", 5, 9, 3), ("uniform", 1, 20, 5), ("uniform", 6, 1, 2),
    ("uniform", 9, 128, 5), ("sparse", 12, 30, 1), ("big_returns", 10, 24, 4), ("no_returns", 8, 40, 5)])
def test_speculative_iterations_edge_instances(vns, kind, K, T, kmax):
    from paper_1704_05132_amd.instances import edge_instance
    inst = edge_instance(kind, K, T, seed=11)
    chains, iters, m = 8, 30, 4
    say(f"  spec_iters edge {kind} {K}x{T} kmax={kmax}")
    with vns.Context(inst, seed=5, chains=chains, k_max=kmax) as ref, \
            vns.Context(inst, seed=5, chains=chains, k_max=kmax, options={vns.OPT_SPEC_ITERS: m}) as ctx:
        ref.run(iters)
        ctx.run(iters)
        assert ctx.stats()["last_run_spec_iters"] == m
        same_search(ctx, ref, chains)
        for g in (0, 3):
            rr = oracle.Chain(inst, 5, g, (1, 2, 4), k_max=kmax).run(iters)
            assert (ctx.trajectory(g) == rr).all(), g


@pytest.mark.parametrize("m", [2, 4, 8])
def test_speculative_iterations_learned_search(vns, m):
    """The learned search (scorer-ranked selection, exact pricing, fallback) with m iterations side by side
    equals the one-workgroup learned search: records, solutions, costs, and the evaluation, neighbourhood
    and fallback counts."""
    inst = workload("plain_100x52")
    chains, iters = 8, 40
    say(f"  learned search, spec_iters m={m}, 100x52 x {chains} chains")
    base = {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: 4}
    with vns.Context(inst, seed=2, chains=chains, options=base) as ref, \
            vns.Context(inst, seed=2, chains=chains, options={**base, vns.OPT_SPEC_ITERS: m}) as ctx:
        for c in (ref, ctx):
            c.mlp_init(21)
        for n in (1, iters):
            ref.run(n)
            ctx.run(n)
            st, rst = ctx.stats(), ref.stats()
            assert st["last_run_spec_iters"] == m and rst["last_run_spec_iters"] == 1
            same_search(ctx, ref, chains)
            for key in ("last_run_learned_evals", "last_run_fallbacks"):
                assert st[key] == rst[key], key
