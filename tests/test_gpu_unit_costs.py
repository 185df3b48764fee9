"""GPU: unit costs p_M, p_R (the parameters Algorithm 1's signature carries) against the oracle, in every
search and pricing path: plain chains, speculative iterations, best-of-G, full and incremental sweeps, and a
batch mixing instances with and without them."""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import draw_instance, workload

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


def with_units(seed, K, T, pM, pR):
    inst = draw_instance(np.random.default_rng([31, seed]), K, T, tag=f"units/{seed}")
    inst.pM = np.full(K, pM, np.int32) if np.isscalar(pM) else np.asarray(pM, np.int32)
    inst.pR = np.full(K, pR, np.int32) if np.isscalar(pR) else np.asarray(pR, np.int32)
    return inst


def same_as_oracle(ctx, g, ref, rr):
    assert (ctx.trajectory(g) == rr).all(), g
    zM, zR = ctx.solution(g)
    assert (zM == ref.zM).all() and (zR == ref.zR).all()
    assert ctx.cost(g) == (ref.F, ref.F_best)


@pytest.mark.parametrize("pM,pR", [(40, 3), (3, 40), (25, 25)])
@pytest.mark.parametrize("mode", ["plain", "spec_iters", "best_of"])
def test_unit_costs_search_equals_oracle(vns, pM, pR, mode):
    inst = with_units(1, 10, 24, pM, pR)
    chains, iters = 4, 30
    opts = {"plain": {}, "spec_iters": {vns.OPT_SPEC_ITERS: 4, vns.OPT_RUN_WAVES: 4},
            "best_of": {vns.OPT_BEST_OF: 3, vns.OPT_RUN_WAVES: 4}}[mode]
    say(f"  unit costs pM={pM} pR={pR}, {mode}")
    with vns.Context(inst, seed=8, chains=chains, options=opts) as ctx:
        ctx.run(iters)
        for g in (0, 3):
            ref = (oracle.BestOfChain(inst, 8, g, (1, 2, 4), 5, G=3) if mode == "best_of"
                   else oracle.Chain(inst, 8, g))
            same_as_oracle(ctx, g, ref, ref.run(iters))


@pytest.mark.parametrize("inc", [0, 1])
def test_unit_costs_sweep_equals_oracle(vns, inc):
    rng = np.random.default_rng(4)
    inst = with_units(2, 12, 52, rng.integers(0, 300, 12), rng.integers(0, 300, 12))
    with vns.Context(inst, seed=3, chains=3, options={vns.OPT_EVAL_INCREMENTAL: inc}) as ctx:
        ctx.run(15)
        r = ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=True)
        n = inst.K * 4 * inst.T
        for g in range(3):
            zM, zR = ctx.solution(g)
            ref, _ = oracle.price_all(inst, zM, zR, 7)
            assert (r["slot_price"][g * n:(g + 1) * n] == ref).all(), g


def test_unit_costs_in_a_mixed_batch(vns):
    insts = [workload("batched_4096", i) for i in range(5)]
    insts[1].pM = np.full(insts[1].K, 30, np.int32)
    insts[1].pR = np.full(insts[1].K, 2, np.int32)
    insts[3].pR = np.full(insts[3].K, 50, np.int32)
    chains, iters = 2, 20
    with vns.Context(insts, seed=6, chains=chains) as ctx:
        ctx.run(iters)
        for i in (0, 1, 3):
            for c in range(chains):
                g = i * chains + c
                ref = oracle.Chain(insts[i], 6, g)
                same_as_oracle(ctx, g, ref, ref.run(iters))


def test_set_unit_costs_recomputes_and_checks(vns):
    inst = draw_instance(np.random.default_rng(9), 6, 12)
    with vns.Context(inst, seed=2, chains=2) as ctx:
        ctx.run(10)
        zM, zR = ctx.solution(1)
        pM, pR = np.full(6, 17, np.int32), np.full(6, 5, np.int32)
        ctx.set_unit_costs(pM, pR)
        inst.pM, inst.pR = pM, pR
        F = oracle.objective(inst, zM, zR)[0]
        assert ctx.cost(1) == (F, F)   # same solution, new objective, best restarts from it
        for bad in ((-1, 0), (0, 1 << 16)):
            with pytest.raises(vns.VNSError):
                ctx.set_unit_costs(np.full(6, bad[0], np.int32), np.full(6, bad[1], np.int32))
