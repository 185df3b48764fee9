"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact (integer costs and indices).

Covers: every slot price of every neighbourhood mask and the per-product / per-instance argmins on random
feasible solutions (T spanning one, several and ragged 32-bit words, K spanning many workgroups); whole GVNS
trajectories (shake, VND, acceptance) for the 10x12 workload and sampled chains of the 100x52 workload at its
full size (64 chains, the launch the benchmark times); batches of uneven instances; degenerate instances;
run(N) + run(M) == run(N + M); set_solution's infeasibility check.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import draw_instance, edge_instance, workload

pytestmark = pytest.mark.gpu
INF = oracle.INF


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


def oracle_product_best(inst, price):
    T = inst.T
    pb, ps = [], []
    for k in range(inst.K):
        v, s = oracle.argmin(price[4 * T * k: 4 * T * (k + 1)])
        pb.append(v)
        ps.append(s)
    return np.array(pb, np.int64), np.array(ps, np.int32)


def check_eval(vns, ctx, inst, chain, zM, zR, masks=(1, 2, 4, 7, 3, 6)):
    for mask in masks:
        say(f"  eval tag={inst.tag} K={inst.K} T={inst.T} chain={chain} mask={mask}")
        got = ctx.eval_neighbourhood(mask, chain)
        ref, n_ref = oracle.price_all(inst, zM, zR, mask)
        assert (got["slot_price"] == ref).all(), np.flatnonzero(got["slot_price"] != ref)[:10]
        pb, ps = oracle_product_best(inst, ref)
        assert (got["prod_best"] == pb).all()
        assert (got["prod_best_slot"] == ps).all()
        v, s = oracle.argmin(ref)
        assert int(got["best"][0]) == v and int(got["best_slot"][0]) == s
        assert ctx.stats()["last_eval_evals"] == n_ref


EVAL_CASES = [("uniform", 1, 1), ("uniform", 3, 2), ("uniform", 7, 12), ("uniform", 5, 31), ("uniform", 5, 32),
              ("uniform", 5, 33), ("uniform", 9, 52), ("uniform", 4, 63), ("uniform", 4, 64), ("uniform", 4, 65),
              ("uniform", 3, 104), ("uniform", 3, 127), ("uniform", 3, 128), ("big_returns", 6, 40),
              ("sparse", 6, 52), ("no_returns", 6, 24), ("returns_eq_demand", 6, 24), ("zero_costs", 4, 20),
              ("zero_demand", 3, 16)]


@pytest.mark.parametrize("kind,K,T", EVAL_CASES)
def test_eval_all_slots_bit_exact(vns, kind, K, T):
    inst = edge_instance(kind, K, T, seed=K * 1000 + T)
    rng = np.random.default_rng([31, K, T])
    with vns.Context(inst, seed=1) as ctx:
        # the initial solution (manufacture every period), then random feasible solutions
        zM = np.ones((K, T), np.uint8)
        zR = np.zeros((K, T), np.uint8)
        check_eval(vns, ctx, inst, 0, zM, zR, masks=(7,))
        for _ in range(3):
            zM, zR = random_solution(inst, rng)
            ctx.set_solution(0, zM, zR)
            F, _ = ctx.cost(0)
            assert F == oracle.objective(inst, zM, zR)[0]
            check_eval(vns, ctx, inst, 0, zM, zR)


def test_eval_workload_instances_all_chains(vns):
    """100x52 workload: 64 chains at distinct solutions, one launch over all chains, every slot checked."""
    inst = workload("plain_100x52")
    rng = np.random.default_rng(32)
    with vns.Context(inst, seed=2, chains=8) as ctx:
        sols = []
        for g in range(8):
            zM, zR = random_solution(inst, rng, p=0.2 + 0.08 * g)
            ctx.set_solution(g, zM, zR)
            sols.append((zM, zR))
        say("  eval all chains 100x52 x8")
        got = ctx.eval_neighbourhood(7, vns.ALL_CHAINS)
        n = 4 * inst.K * inst.T
        for g, (zM, zR) in enumerate(sols):
            ref, _ = oracle.price_all(inst, zM, zR, 7)
            assert (got["slot_price"][g * n:(g + 1) * n] == ref).all(), g
            v, s = oracle.argmin(ref)
            assert int(got["best"][g]) == v and int(got["best_slot"][g]) == s


def test_set_solution_rejects_infeasible(vns):
    inst = workload("plain_10x12")
    with vns.Context(inst, seed=1) as ctx:
        F0 = ctx.cost(0)
        zM = np.zeros((inst.K, inst.T), np.uint8)
        zR = np.zeros((inst.K, inst.T), np.uint8)
        with pytest.raises(vns.VNSError) as e:
            ctx.set_solution(0, zM, zR)
        assert e.value.status == vns.VNS_ERANGE
        assert ctx.cost(0) == F0
        a, b = ctx.solution(0)
        assert a.all() and not b.any()


def compare_chain(ctx, g, ref_chain, rec_gpu, rec_ref, inst):
    assert len(rec_gpu) == len(rec_ref)
    bad = np.flatnonzero(rec_gpu != rec_ref)
    assert len(bad) == 0, (g, bad[:5], rec_gpu[bad[:3]], rec_ref[bad[:3]])
    zM, zR = ctx.solution(g)
    assert (zM == ref_chain.zM).all() and (zR == ref_chain.zR).all()
    F, Fb = ctx.cost(g)
    assert F == ref_chain.F and Fb == ref_chain.F_best


def test_trajectory_10x12_all_500_iterations(vns):
    w = "plain_10x12"
    inst = workload(w)
    say("  run 10x12 x500")
    with vns.Context(inst, seed=1, nb_list=(1, 2)) as ctx:
        ctx.run(500)
        ref = oracle.Chain(inst, 1, 0, (1, 2))
        rr = ref.run(500)
        compare_chain(ctx, 0, ref, ctx.trajectory(0), rr, inst)


@pytest.mark.parametrize("chains_checked,iters", [((0, 17, 63), 30)])
def test_trajectory_100x52_full_launch_sampled_chains(vns, chains_checked, iters):
    """The benchmark's launch shape: 64 chains of the 100x52 instance in one run; sampled chains vs oracle."""
    inst = workload("plain_100x52")
    say(f"  run 100x52 x64 chains x{iters}")
    with vns.Context(inst, seed=2, chains=64) as ctx:
        ctx.run(iters)
        for g in chains_checked:
            ref = oracle.Chain(inst, 2, g)
            rr = ref.run(iters)
            compare_chain(ctx, g, ref, ctx.trajectory(g), rr, inst)
        st = ctx.stats()
        assert st["last_run_evals"] > 0 and st["last_run_ms"] > 0


def test_resume_equals_single_run(vns):
    inst = draw_instance(np.random.default_rng(33), 12, 20)
    say("  resume 12x20")
    with vns.Context(inst, seed=9, chains=3) as a, vns.Context(inst, seed=9, chains=3) as b:
        a.run(40)
        b.run(15)
        r1 = [b.trajectory(g) for g in range(3)]
        b.run(25)
        for g in range(3):
            ra = a.trajectory(g)
            rb = np.concatenate([r1[g], b.trajectory(g)])
            assert (ra[15:] == b.trajectory(g)).all() and (ra[:15] == r1[g]).all() and (ra == rb).all()
            assert a.cost(g) == b.cost(g)
            sa, sb = a.solution(g), b.solution(g)
            assert (sa[0] == sb[0]).all() and (sa[1] == sb[1]).all()


def test_run_is_deterministic(vns):
    inst = workload("plain_10x12")
    say("  determinism")
    recs = []
    for _ in range(2):
        with vns.Context(inst, seed=5, chains=16, nb_list=(1, 2, 4)) as ctx:
            ctx.run(50)
            recs.append(np.concatenate([ctx.trajectory(g) for g in range(16)]))
    assert (recs[0] == recs[1]).all()


@pytest.mark.parametrize("kind,K,T,kmax,nb", [("uniform", 1, 1, 5, (1, 2, 4)), ("zero_demand", 3, 5, 5, (1, 2, 4)),
                                             ("big_returns", 5, 17, 3, (4, 1, 2)), ("sparse", 6, 33, 1, (1, 2, 4)),
                                             ("uniform", 3, 128, 5, (1, 2, 4)), ("uniform", 4, 64, 64, (2, 4)),
                                             ("returns_eq_demand", 5, 9, 7, (1,))])
def test_trajectory_edge_instances(vns, kind, K, T, kmax, nb):
    inst = edge_instance(kind, K, T, seed=7)
    iters = 25
    say(f"  run edge {kind} K={K} T={T} kmax={kmax} nb={nb}")
    with vns.Context(inst, seed=11, chains=2, k_max=kmax, nb_list=nb) as ctx:
        ctx.run(iters)
        for g in range(2):
            ref = oracle.Chain(inst, 11, g, nb, kmax)
            rr = ref.run(iters)
            compare_chain(ctx, g, ref, ctx.trajectory(g), rr, inst)


def test_batch_of_uneven_instances(vns):
    insts = [workload("batched_4096", i) for i in range(4)]
    insts.append(draw_instance(np.random.default_rng(34), 3, 104))
    say("  batch " + " ".join(f"{i.K}x{i.T}" for i in insts))
    chains = 2
    iters = 8
    with vns.Context(insts, seed=3, chains=chains) as ctx:
        ctx.run(iters)
        for i, inst in enumerate(insts):
            for c in range(chains):
                g = i * chains + c
                ref = oracle.Chain(inst, 3, g)
                rr = ref.run(iters)
                compare_chain(ctx, g, ref, ctx.trajectory(g), rr, inst)
        # pricing over the whole batch in one launch
        got = ctx.eval_neighbourhood(7, vns.ALL_CHAINS)
        off = 0
        for i, inst in enumerate(insts):
            for c in range(chains):
                g = i * chains + c
                zM, zR = ctx.solution(g)
                ref, _ = oracle.price_all(inst, zM, zR, 7)
                n = 4 * inst.K * inst.T
                assert (got["slot_price"][off:off + n] == ref).all(), g
                v, s = oracle.argmin(ref)
                assert int(got["best"][g]) == v and int(got["best_slot"][g]) == s
                off += n
