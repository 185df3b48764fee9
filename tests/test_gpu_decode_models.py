"""GPU: the decode readings VNS_OPT_DECODE (strict remanufacture-only shortfall, disposal of unneeded returns,
and both) against the oracle's same readings.

  * every slot price of every chain, at the search's states and at random patterns, at T = 1, 12, 33, 52, 64,
    65, 104 and 128 and on degenerate instances (returns above demand, no returns, sparse demand, zero costs);
  * whole GVNS trajectories, record for record, with the final solutions, in one workgroup per chain and with
    speculative iterations (the cooperative launch), and across several vns_run calls;
  * the per-chain argmins of a batch of uneven instances;
  * the options that do not take another reading (learned search, speculative VND, incremental pricing) are
    refused with VNS_EINVAL, and setting the option restarts every chain from the initial solution.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import edge_instance, random_pattern

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


def with_model(inst, model):
    inst.strict = bool(model & 1)
    inst.dispose = bool(model & 2)
    return inst


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("kind,K,T", [("uniform", 4, 1), ("uniform", 6, 12), ("big_returns", 5, 33),
                                      ("uniform", 5, 52), ("returns_eq_demand", 4, 64), ("big_returns", 3, 65),
                                      ("sparse", 3, 104), ("uniform", 2, 128), ("no_returns", 4, 20),
                                      ("zero_costs", 3, 16)])
def test_prices_and_trajectories(vns, model, kind, K, T):
    inst = with_model(edge_instance(kind, K, T, seed=K * T + model), model)
    chains, iters, seed = 3, 8, 11
    say(f"  decode {model}: {kind} {K}x{T}")
    with vns.Context(inst, seed=seed, chains=chains) as ctx:
        assert ctx.get_option(vns.OPT_DECODE) == model
        # random patterns (seeded generator) on every chain: every slot price
        rng = np.random.default_rng([K, T, model])
        pats = []
        for g in range(chains):
            zM, zR = random_pattern(inst, rng)
            F = oracle.objective(inst, zM, zR)[0]
            if F == oracle.INF:
                with pytest.raises(vns.VNSError) as e:
                    ctx.set_solution(g, zM, zR)
                assert e.value.status == vns.VNS_ERANGE
                zM, zR = np.ones_like(zM), np.zeros_like(zR)
                ctx.set_solution(g, zM, zR)
                F = oracle.objective(inst, zM, zR)[0]
            else:
                ctx.set_solution(g, zM, zR)
            assert ctx.cost(g) == (F, F)
            pats.append((zM, zR))
        out = ctx.eval_neighbourhood(7)
        n = 4 * K * T
        for g, (zM, zR) in enumerate(pats):
            ref, _ = oracle.price_all(inst, zM, zR, 7)
            assert (out["slot_price"][g * n:(g + 1) * n] == ref).all(), g
            assert (int(out["best"][g]), int(out["best_slot"][g])) == oracle.argmin(ref)
    # trajectories from the initial solution, over two calls
    with vns.Context(inst, seed=seed, chains=chains) as ctx:
        ctx.run(iters // 2)
        ctx.run(iters - iters // 2)
        for g in range(chains):
            ref = oracle.Chain(inst, seed, g)
            rr = ref.run(iters)
            assert (ctx.trajectory(g)[-(iters - iters // 2):] == rr[iters // 2:]).all(), g
            zM, zR = ctx.solution(g)
            assert (zM == ref.zM).all() and (zR == ref.zR).all()
            assert ctx.cost(g) == (ref.F, ref.F_best)
            # the search's state: every slot price
            got = ctx.eval_neighbourhood(7, g)["slot_price"]
            assert (got == oracle.price_all(inst, ref.zM, ref.zR, 7)[0]).all()


@pytest.mark.parametrize("model", [1, 2, 3])
def test_speculative_iterations(vns, model):
    inst = with_model(edge_instance("big_returns", 10, 40, seed=model), model)
    chains, iters = 8, 30
    say(f"  decode {model}: speculative iterations, {chains} chains x {iters}")
    with vns.Context(inst, seed=4, chains=chains, options={vns.OPT_SPEC_ITERS: 4, vns.OPT_RUN_WAVES: 4}) as ctx:
        ctx.run(iters)
        assert ctx.stats()["last_run_spec_iters"] == 4
        for g in range(chains):
            ref = oracle.Chain(inst, 4, g)
            assert (ctx.trajectory(g) == ref.run(iters)).all(), g
            zM, zR = ctx.solution(g)
            assert (zM == ref.zM).all() and (zR == ref.zR).all()


@pytest.mark.parametrize("model", [1, 3])
def test_batch_argmins(vns, model):
    insts = [with_model(edge_instance(k, K, T, seed=3), model) for k, K, T in
             (("uniform", 7, 24), ("big_returns", 3, 70), ("uniform", 12, 12), ("sparse", 4, 104))]
    with vns.Context(insts, seed=2, chains=4, options={vns.OPT_EVAL_GROUP: 3}) as ctx:
        ctx.run(5)
        out = ctx.eval_neighbourhood(7, slot_prices=False)
        for g in range(ctx.n_chains):
            inst = insts[g // 4]
            ref = oracle.Chain(inst, 2, g)
            ref.run(5)
            price, _ = oracle.price_all(inst, ref.zM, ref.zR, 7)
            assert (int(out["best"][g]), int(out["best_slot"][g])) == oracle.argmin(price), g


def test_option_rules(vns):
    inst = edge_instance("uniform", 5, 16, seed=1)
    with vns.Context(inst, seed=1, chains=2) as ctx:
        ctx.run(5)
        ctx.set_option(vns.OPT_DECODE, 2)           # restarts every chain from the initial solution
        inst.dispose = True
        ones = np.ones((5, 16), np.uint8)
        F = oracle.objective(inst, ones, np.zeros_like(ones))[0]
        assert ctx.cost(0) == (F, F) and ctx.cost(1) == (F, F)
        with pytest.raises(vns.VNSError) as e:
            ctx.set_option(vns.OPT_DECODE, 4)
        assert e.value.status == vns.VNS_EINVAL
        for opt, val in ((vns.OPT_LEARNED, 100), (vns.OPT_SPECULATE, 1)):
            ctx.set_option(opt, val)
            with pytest.raises(vns.VNSError) as e:
                ctx.run(1)
            assert e.value.status == vns.VNS_EINVAL
            ctx.set_option(opt, 0)
        ctx.set_option(vns.OPT_EVAL_INCREMENTAL, 1)
        with pytest.raises(vns.VNSError) as e:
            ctx.eval_neighbourhood(7, 0)
        assert e.value.status == vns.VNS_EINVAL
        ctx.set_option(vns.OPT_EVAL_INCREMENTAL, 0)
        ctx.run(3)
        ref = oracle.Chain(inst, 1, 0)
        assert (ctx.trajectory(0) == ref.run(3)).all()
