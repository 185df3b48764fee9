"""GPU: the pricing sweep's range form (VNS_OPT_EVAL_SPREAD) against the oracle and the default form.

The range form splits each instance's (chain, product) pairs, product by product, into equal ranges, one
workgroup of 4, 8, 12 or 16 wavefronts each; a range may span several products when their rows fit.  It must
price exactly what the default form prices:
  * every slot price of the 100 x 52 workload's 64 chains at distinct random solutions, against the oracle;
  * a batch of uneven instances (T = 1, 12, 24, 33, 52, 65, 104, 128), with ranges that cross products and
    ranges cut at a product's end, against the oracle and the default form;
  * one chain of a batch, the decode readings, the counted evaluations, the 4096-instance set's argmins;
  * the workgroup table in a caller-bound workspace with stale contents;
  * option rules (values, incremental pricing keeps its own shape).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import draw_instance, edge_instance, workload

pytestmark = pytest.mark.gpu

SPREADS = (4, 8, 12, 16)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vns():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1704_05132_amd import vns as v
    return v


def random_solution(inst, rng, p=0.45):
    zM = (rng.random((inst.K, inst.T)) < p).astype(np.uint8)
    zM[:, 0] = 1
    zR = (rng.random((inst.K, inst.T)) < p / 2).astype(np.uint8)
    return zM, zR


def set_random(ctx, insts, chains, rng):
    """Distinct random feasible solutions on every chain; returns them per chain."""
    sols = []
    for g in range(ctx.n_chains):
        inst = insts[g // chains]
        while True:
            zM, zR = random_solution(inst, rng, p=0.15 + 0.6 * rng.random())
            if oracle.objective(inst, zM, zR)[0] != oracle.INF:
                break
        ctx.set_solution(g, zM, zR)
        sols.append((zM, zR))
    return sols


def eval_with(vns, ctx, spread, mask=7, chain=None):
    ctx.set_option(vns.OPT_EVAL_SPREAD, spread)
    assert ctx.get_option(vns.OPT_EVAL_SPREAD) == spread
    out = ctx.eval_neighbourhood(mask, vns.ALL_CHAINS if chain is None else chain)
    return out, ctx.stats()["last_eval_evals"]


def check_against_oracle(out, insts, chains, sols, mask, gs=None):
    off = 0
    gs = range(len(sols)) if gs is None else gs
    for i, g in enumerate(gs):
        inst = insts[g // chains]
        zM, zR = sols[g]
        ref, _ = oracle.price_all(inst, zM, zR, mask)
        n = 4 * inst.K * inst.T
        assert (out["slot_price"][off:off + n] == ref).all(), (g, np.flatnonzero(out["slot_price"][off:off + n] != ref)[:8])
        v, s = oracle.argmin(ref)
        assert int(out["best"][i]) == v and int(out["best_slot"][i]) == s, g
        off += n


def same(a, b):
    for k in ("slot_price", "prod_best", "prod_best_slot", "best", "best_slot"):
        if a[k] is not None:
            assert (a[k] == b[k]).all(), k


@pytest.mark.parametrize("spread", SPREADS)
def test_workload_100x52_every_slot(vns, spread):
    inst = workload("plain_100x52")
    chains = 64
    rng = np.random.default_rng([51, spread])
    with vns.Context(inst, seed=2, chains=chains) as ctx:
        sols = set_random(ctx, [inst], chains, rng)
        say(f"  range form {spread} wavefronts: 100x52 x {chains} chains")
        out, n = eval_with(vns, ctx, spread)
        check_against_oracle(out, [inst], chains, sols, 7)
        base, n0 = eval_with(vns, ctx, 0)
        same(out, base)
        assert n == n0


def uneven_batch():
    insts = [edge_instance("uniform", 9, 1, seed=1), edge_instance("uniform", 7, 12, seed=2),
             edge_instance("big_returns", 11, 24, seed=3), edge_instance("sparse", 5, 33, seed=4),
             workload("batched_4096", 3), edge_instance("uniform", 4, 65, seed=5),
             draw_instance(np.random.default_rng(34), 3, 104), edge_instance("uniform", 3, 128, seed=6),
             edge_instance("no_returns", 6, 20, seed=7)]
    return insts


@pytest.mark.parametrize("spread", SPREADS)
@pytest.mark.parametrize("mask", [7, 1, 6])
def test_uneven_batch(vns, spread, mask):
    insts = uneven_batch()
    chains = 3
    rng = np.random.default_rng([52, spread, mask])
    with vns.Context(insts, seed=5, chains=chains) as ctx:
        sols = set_random(ctx, insts, chains, rng)
        say(f"  range form {spread}: batch " + " ".join(f"{i.K}x{i.T}" for i in insts) + f" mask {mask}")
        out, n = eval_with(vns, ctx, spread, mask)
        check_against_oracle(out, insts, chains, sols, mask)
        base, n0 = eval_with(vns, ctx, 0, mask)
        same(out, base)
        assert n == n0


@pytest.mark.parametrize("spread", SPREADS)
def test_after_search_and_one_chain(vns, spread):
    insts = uneven_batch()
    chains = 4
    with vns.Context(insts, seed=7, chains=chains) as ctx:
        ctx.run(6)
        sols = [ctx.solution(g) for g in range(ctx.n_chains)]
        out, _ = eval_with(vns, ctx, spread)
        check_against_oracle(out, insts, chains, sols, 7)
        for g in (0, 5, 17, ctx.n_chains - 1):
            one, _ = eval_with(vns, ctx, spread, chain=g)
            check_against_oracle(one, insts, chains, sols, 7, gs=[g])


@pytest.mark.parametrize("model", [1, 2, 3])
def test_decode_readings(vns, model):
    insts = uneven_batch()
    for inst in insts:
        inst.strict = bool(model & 1)
        inst.dispose = bool(model & 2)
    chains = 2
    with vns.Context(insts, seed=9, chains=chains) as ctx:
        assert ctx.get_option(vns.OPT_DECODE) == model
        ctx.run(5)
        sols = [ctx.solution(g) for g in range(ctx.n_chains)]
        base, n0 = eval_with(vns, ctx, 0)
        for spread in SPREADS:
            out, n = eval_with(vns, ctx, spread)
            same(out, base)
            assert n == n0
        check_against_oracle(base, insts, chains, sols, 7)


def test_batched_4096_argmins(vns):
    insts = [workload("batched_4096", i) for i in range(4096)]
    with vns.Context(insts, seed=3, chains=8) as ctx:
        ctx.run(3)
        say("  range form: 4096 instances x 8 chains, argmins against the default form")
        base = ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False)
        n0 = ctx.stats()["last_eval_evals"]
        for spread in SPREADS:
            ctx.set_option(vns.OPT_EVAL_SPREAD, spread)
            out = ctx.eval_neighbourhood(7, vns.ALL_CHAINS, slot_prices=False)
            same(out, base)
            assert ctx.stats()["last_eval_evals"] == n0
        # sampled chains against the oracle
        for g in (0, 12345, 8 * 4096 - 1):
            inst = insts[g // 8]
            zM, zR = ctx.solution(g)
            ref, _ = oracle.price_all(inst, zM, zR, 7)
            assert (int(out["best"][g]), int(out["best_slot"][g])) == oracle.argmin(ref)


def test_option_rules(vns):
    inst = edge_instance("uniform", 5, 16, seed=1)
    with vns.Context(inst, seed=1, chains=3) as ctx:
        assert ctx.get_option(vns.OPT_EVAL_SPREAD) == 0
        for v in (-1, 1, 2, 5, 32):
            with pytest.raises(vns.VNSError) as e:
                ctx.set_option(vns.OPT_EVAL_SPREAD, v)
            assert e.value.status == vns.VNS_EINVAL
        ctx.run(4)
        base = ctx.eval_neighbourhood(7)
        # incremental pricing keeps its own launch shape; the prices are the same
        ctx.set_option(vns.OPT_EVAL_SPREAD, 16)
        ctx.set_option(vns.OPT_EVAL_INCREMENTAL, 1)
        same(ctx.eval_neighbourhood(7), base)
        ctx.set_option(vns.OPT_EVAL_INCREMENTAL, 0)
        same(ctx.eval_neighbourhood(7), base)


@pytest.mark.parametrize("spread", [4, 16])
def test_bound_workspace(vns, spread):
    """The range form's workgroup table in a caller-bound workspace (stale contents) equals own buffers."""
    import torch
    insts = uneven_batch()
    chains = 3
    with vns.Context(insts, seed=8, chains=chains) as a, vns.Context(insts, seed=8, chains=chains) as b:
        for ctx in (a, b):
            ctx.bind_stream(torch.cuda.current_stream())
            ctx.run(5)
            ctx.set_option(vns.OPT_EVAL_SPREAD, spread)
        flags = vns.WS_EVAL_PRICES
        buf = torch.empty(b.workspace_bytes(flags), dtype=torch.uint8, device="cuda")
        b.bind_workspace(buf, flags)
        buf.fill_(0x5A)
        torch.cuda.synchronize()
        ea, eb = a.eval_neighbourhood(7), b.eval_neighbourhood(7)
        for k in ea:
            assert (ea[k] == eb[k]).all(), k
        oa, ob = a.eval_neighbourhood(6, 7), b.eval_neighbourhood(6, 7)
        for k in oa:
            assert (oa[k] == ob[k]).all(), k
        b.bind_workspace(None, 0)
