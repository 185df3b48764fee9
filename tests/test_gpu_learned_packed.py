"""GPU: the packed learned VND (VNS_OPT_LEARNED_PACK) against the one-product learned VND.

The packed form runs the learned VNDs of up to P products in lockstep, all of a workgroup's wavefronts
together, and prices their selections, and then their fallbacks, in shared passes.  Per product it must take
exactly the same steps: so every record, solution and cost, and the counted exact evaluations, neighbourhood
evaluations and fallbacks, equal the one-product search's (which the other learned tests check against the
oracle's selection and fallback rules and local optimality).  Covered: P = 2, 3, 8; 1, 2 and 4 wavefronts; rows resident in LDS or
staged per product; T <= 64 and T > 64; the memo of unchanged neighbourhoods; a selection of every move
(permille 1000); speculative iterations; the first iteration (every product of x); uneven batches of
instances; degenerate instances (one product, T = 1, no returns).
"""
import sys

import numpy as np
import pytest

from oracle import learned as L
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


def params(seed):
    rng = np.random.default_rng(seed)
    ps = L.init_params(seed)
    ps[1] = rng.normal(0, 0.2, 64).astype(np.float32)
    ps[3] = rng.normal(0, 0.2, 64).astype(np.float32)
    ps[5] = np.float32([0.3])
    return ps


def run_pair(vns, insts, chains, iters_list, opts, pack, seed=3, pseed=61):
    """The same learned search one product at a time and packed; returns both contexts' observations."""
    out = []
    for p in (0, pack):
        o = dict(opts)
        o[vns.OPT_LEARNED_PACK] = p
        with vns.Context(insts if len(insts) > 1 else insts[0], seed=seed, chains=chains, options=o) as ctx:
            ctx.mlp_set(params(pseed))
            st_all = []
            for it in iters_list:
                ctx.run(it)
                st = ctx.stats()
                st_all.append((st["last_run_evals"], st["last_run_learned_evals"], st["last_run_fallbacks"],
                               st["last_run_spec_iters"]))
            sols = [ctx.solution(g) for g in range(ctx.n_chains)]
            out.append({"traj": [ctx.trajectory(g) for g in range(ctx.n_chains)], "sols": sols,
                        "costs": ctx.costs(), "stats": st_all})
    return out


def assert_same(a, b):
    for g, (ta, tb) in enumerate(zip(a["traj"], b["traj"])):
        assert (ta == tb).all(), g
    for g, ((ma, ra), (mb, rb)) in enumerate(zip(a["sols"], b["sols"])):
        assert (ma == mb).all() and (ra == rb).all(), g
    assert (a["costs"][0] == b["costs"][0]).all() and (a["costs"][1] == b["costs"][1]).all()
    assert a["stats"] == b["stats"], (a["stats"], b["stats"])


@pytest.mark.parametrize("pack,waves", [(2, 1), (3, 2), (8, 4), (8, 1)])
@pytest.mark.parametrize("kind,K,T", [("uniform", 12, 24), ("big_returns", 9, 52), ("sparse", 5, 104),
                                      ("uniform", 6, 128)])
def test_packed_equals_one_product(vns, pack, waves, kind, K, T):
    insts = [edge_instance(kind, K, T, seed=K + T)]
    say(f"  packed learned VND P={pack} waves={waves} {kind} {K}x{T}")
    a, b = run_pair(vns, insts, 3, (1, 7), {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: waves}, pack)
    assert a["stats"][0][1] > 0
    assert_same(a, b)


@pytest.mark.parametrize("lds", [0, 65536])
@pytest.mark.parametrize("memo", [0, 1])
def test_packed_rows_staged_or_resident_and_memo(vns, lds, memo):
    insts = [workload("learned_100x52", 0)]
    say(f"  packed learned VND, rows lds={lds} memo={memo}")
    opts = {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: 2, vns.OPT_RUN_LDS: lds, vns.OPT_VND_MEMO: memo}
    a, b = run_pair(vns, insts, 4, (1, 5), opts, 4)
    assert_same(a, b)


def test_packed_every_move_selected(vns):
    insts = [edge_instance("uniform", 7, 33, seed=2)]
    a, b = run_pair(vns, insts, 2, (1, 6), {vns.OPT_LEARNED: 1000, vns.OPT_RUN_WAVES: 2}, 5)
    assert a["stats"][1][2] == 0 or a["stats"][1][2] > 0   # the fallback can still be taken (nothing improves)
    assert_same(a, b)


def test_packed_batch_of_uneven_instances(vns):
    insts = [edge_instance(k, K, T, seed=5) for k, K, T in
             (("uniform", 7, 24), ("big_returns", 3, 70), ("uniform", 12, 12), ("sparse", 4, 104))]
    a, b = run_pair(vns, insts, 3, (1, 8), {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: 2}, 3)
    assert_same(a, b)


@pytest.mark.parametrize("kind,K,T", [("uniform", 1, 20), ("uniform", 6, 1), ("no_returns", 5, 30),
                                      ("zero_costs", 4, 16)])
def test_packed_degenerate_instances(vns, kind, K, T):
    insts = [edge_instance(kind, K, T, seed=7)]
    a, b = run_pair(vns, insts, 2, (1, 6), {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: 2}, 4)
    assert_same(a, b)


@pytest.mark.parametrize("m", [2, 8])
def test_packed_speculative_iterations(vns, m):
    insts = [workload("learned_100x52", 1)]
    say(f"  packed learned VND with {m} speculative iterations")
    opts = {vns.OPT_LEARNED: 100, vns.OPT_RUN_WAVES: 4, vns.OPT_SPEC_ITERS: m}
    a, b = run_pair(vns, insts, 8, (1, 12), opts, 4)
    assert a["stats"][1][3] == m and b["stats"][1][3] == m
    assert_same(a, b)


def test_pack_option_range(vns):
    with vns.Context(edge_instance("uniform", 3, 8, seed=1), seed=1) as ctx:
        for v in (0, 1, 2, 8):
            ctx.set_option(vns.OPT_LEARNED_PACK, v)
            assert ctx.get_option(vns.OPT_LEARNED_PACK) == v
        for v in (-1, 9):
            with pytest.raises(vns.VNSError) as e:
                ctx.set_option(vns.OPT_LEARNED_PACK, v)
            assert e.value.status == vns.VNS_EINVAL
