"""GPU: the move log (training records the search writes for the learned scorer) against the oracle.

For a plain search logging its moves, the test replays the same GVNS iterations with the oracle's own steps
(Shake with the same Philox draws, the VND of Algorithm 1 with its move trace, accept if better) and
derives every record the log must hold:
  * one record per applied move: the 16 features of that move (oracle.learned.move_features) with respect to
    the product's pattern just before it, and the target (cost after - cost before) / 1000 in float32;
  * at most one contrast record per applied move: a priced move of the same evaluation, so its features and
    target are those of some valid move of the same neighbourhood at the same pattern (its price from
    oracle.price_all) that is not the applied one.
The log's order depends on scheduling, so records are compared as multisets.  Checked at T = 16 (one setup
word), T = 70 (a ragged second word) and T = 104 (four words), with several chains.
"""
import sys
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import learned as ol
from paper_1704_05132_amd.instances import edge_instance

pytestmark = pytest.mark.gpu

NB = (1, 2, 4)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vns():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1704_05132_amd import vns as v
    return v


def _key(f, y):
    return (tuple(np.asarray(f, np.float32).view(np.uint32).tolist()), int(np.float32(y).view(np.uint32)))


def expected_records(inst, seed, chain, iters, k_max=5):
    """(applied records, per applied move the set of admissible contrast records) of `iters` GVNS
    iterations of one chain, from the oracle's shake, traced VND and acceptance rule."""
    zM = np.ones((inst.K, inst.T), np.uint8)
    zR = np.zeros((inst.K, inst.T), np.uint8)
    F = oracle.objective(inst, zM, zR)[0]
    k = 1
    applied, contrast_sets = [], []
    for it in range(iters):
        sM, sR, _ = oracle.shake(inst, zM, zR, k, seed, chain, it)
        F_local, vM, vR, _, trace = oracle.vnd(inst, sM, sR, NB, trace=True)
        # replay the trace product by product from the shaken pattern
        cur_M, cur_R = sM.copy(), sR.copy()
        F_prev = oracle.objective(inst, sM, sR)[0]
        for _, nb, p, slot, F_after in trace:
            p, slot = int(p), int(slot)
            rowM, rowR = cur_M[p].copy(), cur_R[p].copy()
            f = ol.move_features(inst, p, rowM, rowR, slot)
            dc = int(F_after) - F_prev
            applied.append(_key(f, np.float32(dc) / np.float32(1000)))
            # every other priced move of the same neighbourhood of product p at this pattern
            one = inst.product(p)
            prices, _ = oracle.price_all(one, rowM[None, :], rowR[None, :], int(nb))
            c_before = oracle.objective(one, rowM[None, :], rowR[None, :])[0]
            opts = set()
            for l in np.nonzero(prices != oracle.INF)[0]:
                if int(l) == slot:
                    continue
                fl = ol.move_features(inst, p, rowM, rowR, int(l))
                opts.add(_key(fl, np.float32(int(prices[l]) - c_before) / np.float32(1000)))
            contrast_sets.append(opts)
            ok, nM, nR = oracle.apply_slot(inst.T, rowM, rowR, slot)
            assert ok
            cur_M[p], cur_R[p] = nM, nR
            F_prev = int(F_after)
        assert (cur_M == vM).all() and (cur_R == vR).all() and F_prev == F_local
        if F_local < F:
            zM, zR, F, k = vM, vR, F_local, 1
        else:
            k = 1 if k >= k_max else k + 1
    return applied, contrast_sets


@pytest.mark.parametrize("K,T,iters,chains", [(5, 16, 4, 3), (3, 70, 3, 2), (2, 104, 3, 2)])
def test_move_log_matches_oracle(vns, K, T, iters, chains):
    inst = edge_instance("uniform", K, T, seed=K + T)
    seed = 17
    say(f"  move log: K={K} T={T}, {chains} chains x {iters} iterations")
    with vns.Context(inst, seed=seed, chains=chains, options={vns.OPT_LOG: 100000}) as ctx:
        ctx.run(iters)
        X, y = ctx.move_log()
    got = Counter(_key(X[i], y[i]) for i in range(len(y)))
    want_applied = Counter()
    contrast_sets = []
    for g in range(chains):
        a, cs = expected_records(inst, seed, g, iters)
        want_applied.update(a)
        contrast_sets += cs
    n_applied = sum(want_applied.values())
    say(f"    {len(y)} records, {n_applied} applied moves")
    assert n_applied > 0
    # every applied move is logged with its exact features and target
    for key, n in want_applied.items():
        assert got[key] >= n, key
    rest = got - want_applied
    n_contrast = sum(rest.values())
    assert n_applied <= len(y) <= 2 * n_applied
    assert n_contrast == len(y) - n_applied
    # each remaining record is a priced, non-applied move of the evaluation of some applied move
    union = set().union(*contrast_sets) if contrast_sets else set()
    for key in rest:
        assert key in union, key
    assert n_contrast > 0
