"""GPU: the boundary's status codes, the best-solution query and the caller-owned workspace, through the C ABI.

  * VNS_ENOMEM from a failed device allocation (forced from the host with vns_test_inject_failure, no real
    shortage), at creation and inside a later call, which leaves the context usable;
  * VNS_EDEVICE (a HIP failure reported by the injection hook, no device fault), after which every call but
    vns_destroy and vns_last_error returns VNS_ESTATE;
  * vns_get_solution(..., VNS_SOLUTION_BEST): the best solution of Algorithm 2's search.  Under the
    accept-if-better rule it is the current one; in best-of-G as printed (the selected result always replaces
    x) it is tracked apart, and equals the first solution of the lowest objective in the oracle's run;
  * a bound workspace gives the same prices, argmins and trajectories as the context's own buffers, and a
    workspace too small, badly aligned, or outgrown after an option change is refused with VNS_EINVAL;
  * vns_set_solution of an infeasible pattern returns VNS_ERANGE and leaves x as it was.
"""
import ctypes
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


@pytest.fixture(autouse=True)
def _clear_injection(vns):
    yield
    vns.inject_failure(vns.INJECT_ALLOC, 0)
    vns.inject_failure(vns.INJECT_DEVICE, 0)


def test_enomem_at_create_and_in_a_call(vns):
    inst = edge_instance("uniform", 6, 10, seed=1)
    say("  ENOMEM: create with the first device allocation failing")
    vns.inject_failure(vns.INJECT_ALLOC, 1)
    with pytest.raises(vns.VNSError) as e:
        vns.Context(inst, seed=1)
    assert e.value.status == vns.VNS_ENOMEM
    assert b"memory" in vns.lib().vns_last_error(None).lower()
    say("  ENOMEM: a move-log allocation failing inside vns_set_option")
    with vns.Context(inst, seed=1, chains=2) as ctx:
        vns.inject_failure(vns.INJECT_ALLOC, 1)
        with pytest.raises(vns.VNSError) as e:
            ctx.set_option(vns.OPT_LOG, 1000)
        assert e.value.status == vns.VNS_ENOMEM
        # the context is still live and exact
        ctx.run(6)
        for g in range(2):
            ref = oracle.Chain(inst, 1, g)
            assert (ctx.trajectory(g) == ref.run(6)).all()


def test_edevice_then_estate(vns):
    inst = edge_instance("uniform", 6, 10, seed=2)
    ctx = vns.Context(inst, seed=3)
    ctx.run(2)
    say("  EDEVICE: the next call reports a HIP failure")
    vns.inject_failure(vns.INJECT_DEVICE, 1)
    with pytest.raises(vns.VNSError) as e:
        ctx.run(1)
    assert e.value.status == vns.VNS_EDEVICE
    assert b"injected" in vns.lib().vns_last_error(ctx.h)
    for call in (lambda: ctx.run(1), lambda: ctx.cost(0), lambda: ctx.eval_neighbourhood(7, 0),
                 lambda: ctx.solution(0), lambda: ctx.set_option(vns.OPT_KMAX, 3)):
        with pytest.raises(vns.VNSError) as e:
            call()
        assert e.value.status == vns.VNS_ESTATE
    ctx.close()   # vns_destroy is still valid


def test_best_solution_under_accept_if_better_is_current(vns):
    inst = workload("plain_10x12")
    with vns.Context(inst, seed=1, chains=3, nb_list=(1, 2)) as ctx:
        ctx.run(40)
        F, Fb = ctx.costs()
        for g in range(3):
            zM, zR = ctx.solution(g)
            bM, bR = ctx.solution(g, vns.SOLUTION_BEST)
            assert (zM == bM).all() and (zR == bR).all()
            assert F[g] == Fb[g] == oracle.objective(inst, bM, bR)[0]
        with pytest.raises(vns.VNSError) as e:
            ctx.solution(0, 2)
        assert e.value.status == vns.VNS_EINVAL


@pytest.mark.parametrize("G", [3, 4])
def test_best_solution_of_best_of_g_as_printed(vns, G):
    """Best-of-G as printed moves x to the selected result even when it is worse; the best solution is the
    first one that reached the lowest objective, as the oracle's chain run one iteration at a time shows."""
    inst = edge_instance("uniform", 10, 16, seed=7)
    chains, iters = 4, 40
    say(f"  best solution, best-of-{G} as printed: {chains} chains x {iters} iterations")
    with vns.Context(inst, seed=8, chains=chains, options={vns.OPT_BEST_OF: G, vns.OPT_BEST_OF_LITERAL: 1,
                                                           vns.OPT_RUN_WAVES: 4}) as ctx:
        ctx.run(iters // 2)
        ctx.run(iters - iters // 2)   # tracked across calls
        diverged = 0
        for g in range(chains):
            ref = oracle.BestOfChain(inst, 8, g, (1, 2, 4), 5, G=G, literal=True)
            bestF, bM, bR = ref.F, ref.zM.copy(), ref.zR.copy()
            for _ in range(iters):
                ref.run(1)
                if ref.F < bestF:
                    bestF, bM, bR = ref.F, ref.zM.copy(), ref.zR.copy()
            assert ref.F_best == bestF
            gM, gR = ctx.solution(g, vns.SOLUTION_BEST)
            assert (gM == bM).all() and (gR == bR).all(), g
            assert ctx.cost(g) == (ref.F, ref.F_best)
            cM, cR = ctx.solution(g)
            assert (cM == ref.zM).all() and (cR == ref.zR).all()
            diverged += int(ref.F != ref.F_best)
        say(f"    chains whose x is worse than their best: {diverged}")


def test_workspace_matches_own_buffers(vns):
    import torch
    inst = edge_instance("uniform", 9, 70, seed=4)   # two setup words, ragged
    chains, iters = 8, 25
    opts = {vns.OPT_SPEC_ITERS: 4, vns.OPT_RUN_WAVES: 4}
    say("  workspace: own buffers vs a bound torch buffer (pricing and speculative iterations)")
    with vns.Context(inst, seed=5, chains=chains, options=opts) as a, \
            vns.Context(inst, seed=5, chains=chains, options=opts) as b:
        flags = vns.WS_RUN | vns.WS_EVAL_PRICES
        need = b.workspace_bytes(flags)
        assert need >= b.workspace_bytes(vns.WS_EVAL) > 0 and b.workspace_bytes(0) == 0
        buf = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
        b.bind_stream(torch.cuda.current_stream())
        a.bind_stream(torch.cuda.current_stream())
        # refused: too small, misaligned, unknown flags
        L = vns.lib()
        assert L.vns_bind_workspace(b.h, ctypes.c_void_p(buf.data_ptr()), need - 1, flags) == vns.VNS_EINVAL
        assert L.vns_bind_workspace(b.h, ctypes.c_void_p(buf.data_ptr() + 128), need, flags) == vns.VNS_EINVAL
        assert L.vns_bind_workspace(b.h, ctypes.c_void_p(buf.data_ptr()), need, 8) == vns.VNS_EINVAL
        b.bind_workspace(buf, flags)
        buf.fill_(0xA5)   # stale contents must not matter
        torch.cuda.synchronize()
        for ctx in (a, b):
            ctx.run(iters)
        assert b.stats()["last_run_spec_iters"] == a.stats()["last_run_spec_iters"] == 4
        for g in range(chains):
            assert (a.trajectory(g) == b.trajectory(g)).all()
        ea, eb = a.eval_neighbourhood(7), b.eval_neighbourhood(7)
        for k in ea:
            assert (ea[k] == eb[k]).all(), k
        one_a, one_b = a.eval_neighbourhood(5, 3), b.eval_neighbourhood(5, 3)
        for k in one_a:
            assert (one_a[k] == one_b[k]).all(), k
        # against the oracle too, at the oracle's own state of chain 3 (which the device's equals)
        ch = oracle.Chain(inst, 5, 3)
        ch.run(iters)
        zM, zR = b.solution(3)
        assert (zM == ch.zM).all() and (zR == ch.zR).all()
        ref, _ = oracle.price_all(inst, ch.zM, ch.zR, 5)
        assert (one_b["slot_price"] == ref).all()
        # more speculative iterations outgrow the bound buffer: refused without running
        b.set_option(vns.OPT_SPEC_ITERS, 8)
        assert b.workspace_bytes(flags) > need + 4096
        with pytest.raises(vns.VNSError) as e:
            b.run(5)
        assert e.value.status == vns.VNS_EINVAL
        # unbinding returns to the context's own buffers
        b.bind_workspace(None, 0)
        a.set_option(vns.OPT_SPEC_ITERS, 8)
        a.run(10)
        b.run(10)
        for g in range(chains):
            assert (a.trajectory(g) == b.trajectory(g)).all()


def test_set_solution_infeasible_leaves_x(vns):
    inst = edge_instance("uniform", 5, 8, seed=9)
    with vns.Context(inst, seed=2, chains=1) as ctx:
        ctx.run(10)
        zM, zR = ctx.solution(0)
        F = ctx.cost(0)[0]
        bad_M = np.zeros_like(zM)   # no manufacturing setup at all: demand before any setup is infeasible
        bad_R = np.zeros_like(zR)
        assert inst.D.sum() > 0
        with pytest.raises(vns.VNSError) as e:
            ctx.set_solution(0, bad_M, bad_R)
        assert e.value.status == vns.VNS_ERANGE
        z2M, z2R = ctx.solution(0)
        assert (z2M == zM).all() and (z2R == zR).all()
        assert ctx.cost(0) == (F, F)
