"""GPU: the allocation-free pricing call (vns_eval_neighbourhood_noalloc) against vns_eval_neighbourhood.

Through the C ABI, on two calls in a row (the second with a smaller input), the outputs must be identical to
the allocating call's: per-product best prices and slots, per-chain argmins, every slot price, and the counted
move-evaluations.  Also: a batch of uneven instances priced in ragged groups of chains, two contexts sharing
the GPU's scratch one after the other, and a request beyond the static scratch refused with VNS_EINVAL.
"""
import sys

import numpy as np
import pytest

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


def same(ctx, nb, chain, slot_prices, prod_best=True):
    ref = ctx.eval_neighbourhood(nb, chain, slot_prices=slot_prices, prod_best=prod_best)
    ev_ref = ctx.stats()["last_eval_evals"]
    got = ctx.eval_neighbourhood_noalloc(nb, chain, slot_prices=slot_prices, prod_best=prod_best)
    ev_got = ctx.stats()["last_eval_evals"]
    for k, v in ref.items():
        if v is None:
            assert got[k] is None
        else:
            assert (got[k] == v).all(), (k, nb, chain)
    assert ev_got == ev_ref > 0
    return got


def test_noalloc_equals_allocating_call_twice_smaller_second(vns):
    inst = workload("plain_100x52")
    with vns.Context(inst, seed=2, chains=64, options={vns.OPT_EVAL_GROUP: 5}) as ctx:
        ctx.run(30)
        say("  noalloc: all 64 chains (argmins), then one chain with every slot price")
        same(ctx, 7, vns.ALL_CHAINS, slot_prices=False)
        same(ctx, 7, 37, slot_prices=True)
        same(ctx, 4, 3, slot_prices=True, prod_best=False)
        # beyond the static scratch: every slot of 64 chains of 100 x 52 is 10.6 MB
        with pytest.raises(vns.VNSError) as e:
            ctx.eval_neighbourhood_noalloc(7, vns.ALL_CHAINS, slot_prices=True)
        assert e.value.status == vns.VNS_EINVAL
        # still usable after the refusal
        same(ctx, 2, 63, slot_prices=True)


def test_noalloc_batch_ragged_groups_and_two_contexts(vns):
    insts = [edge_instance("uniform", 3, 1, seed=1), edge_instance("uniform", 5, 12, seed=2),
             edge_instance("big_returns", 2, 70, seed=3), edge_instance("sparse", 4, 104, seed=4),
             edge_instance("uniform", 6, 128, seed=5)]
    with vns.Context(insts, seed=9, chains=5, options={vns.OPT_EVAL_GROUP: 3}) as a, \
            vns.Context(insts[1], seed=4, chains=3) as b:
        a.run(6)
        b.run(4)
        say("  noalloc: a batch of 5 uneven instances x 5 chains in groups of 3, then another context")
        same(a, 7, vns.ALL_CHAINS, slot_prices=True)
        same(b, 7, vns.ALL_CHAINS, slot_prices=True)
        same(a, 5, 17, slot_prices=True)
        same(b, 1, 2, slot_prices=False)
