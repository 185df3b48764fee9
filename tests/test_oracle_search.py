"""Pins of the oracle's search layer (CPU only): VND (Algorithm 1), shake and GVNS (Algorithm 2).

  * VND: the result is a local optimum of every neighbourhood in its list (checked with the pinned slot
    prices), the objective never rises, and product independence (Section 3): VND on K products equals VND
    on each one-product instance.
  * shake: the flips are the ones derived from numpy.random.Philox outputs with the multiply-shift map, and
    an applied flip never leaves its product infeasible.
  * GVNS: the acceptance rule, the k schedule, best tracking and run(N) + run(M) == run(N + M).
"""
import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import draw_instance, edge_instance, workload

INF = oracle.INF


def _random_solution(inst, rng, p=0.5):
    zM = (rng.random((inst.K, inst.T)) < p).astype(np.uint8)
    zM[:, 0] = 1
    zR = (rng.random((inst.K, inst.T)) < p / 2).astype(np.uint8)
    return zM, zR


@pytest.mark.parametrize("nb_list", [(1, 2), (1, 2, 4), (4, 1), (2,)])
@pytest.mark.parametrize("seed", range(3))
def test_vnd_reaches_local_optimum(nb_list, seed):
    rng = np.random.default_rng([21, seed])
    inst = draw_instance(rng, 6, 13)
    zM, zR = _random_solution(inst, rng)
    F0, _ = oracle.objective(inst, zM, zR)
    F, a, b, ev = oracle.vnd(inst, zM, zR, nb_list)
    assert F <= F0
    assert oracle.objective(inst, a, b)[0] == F
    mask = 0
    for nb in nb_list:
        mask |= nb
    price, _ = oracle.price_all(inst, a, b, mask)
    assert price.min() >= F                      # no strictly improving move is left
    assert ev > 0


def test_vnd_from_initial_solution_all_workload_sizes():
    for name in ("plain_10x12",):
        inst = workload(name)
        zM = np.ones((inst.K, inst.T), np.uint8)
        zR = np.zeros_like(zM)
        F0, _ = oracle.objective(inst, zM, zR)
        F, a, b, _ = oracle.vnd(inst, zM, zR, (1, 2))
        assert F < F0
        price, _ = oracle.price_all(inst, a, b, 3)
        assert price.min() >= F


@pytest.mark.parametrize("seed", range(3))
def test_vnd_is_separable_by_product(seed):
    rng = np.random.default_rng([22, seed])
    inst = draw_instance(rng, 5, 9)
    zM, zR = _random_solution(inst, rng)
    F, a, b, _ = oracle.vnd(inst, zM, zR, (1, 2, 4))
    for k in range(inst.K):
        sub = inst.product(k)
        Fk, ak, bk, _ = oracle.vnd(sub, zM[k:k + 1], zR[k:k + 1], (1, 2, 4))
        assert (ak == a[k:k + 1]).all() and (bk == b[k:k + 1]).all()


def _counter_minus_one(ctr):
    """numpy's Philox produces block(counter + 1): return counter - 1 as a 256-bit little-endian integer."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    return np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], np.uint64)


def _numpy_draw(seed, chain, it, j, n):
    bg = np.random.Philox(key=np.array([seed, chain], np.uint64), counter=_counter_minus_one([it, j, 0, 0]))
    o0 = int(bg.random_raw(1)[0])
    return ((o0 >> 32) * n) >> 32


@pytest.mark.parametrize("seed,chain,it", [(1, 0, 0), (2, 17, 1999), (3, 5, 7), (9, 63, 123456)])
def test_shake_draws_match_numpy_philox(seed, chain, it):
    inst = workload("plain_10x12")
    n = 2 * inst.K * inst.T
    for j in range(6):
        assert oracle.draw(seed, chain, it, j, n) == _numpy_draw(seed, chain, it, j, n)


@pytest.mark.parametrize("kind", ["uniform", "sparse", "big_returns"])
@pytest.mark.parametrize("it", range(8))
def test_shake_applies_the_drawn_feasible_flips(kind, it):
    inst = edge_instance(kind, 4, 7, seed=it)
    rng = np.random.default_rng([23, it])
    zM, zR = _random_solution(inst, rng, 0.4)
    T, n = inst.T, 2 * inst.K * inst.T
    k = 1 + it % 5
    a, b, applied = oracle.shake(inst, zM, zR, k, 5, 3, it)
    em, er = zM.copy(), zR.copy()
    for j in range(k):
        f = _numpy_draw(5, 3, it, j, n)
        p, r = divmod(f, 2 * T)
        row = em if r < T else er
        t = r if r < T else r - T
        row[p, t] ^= 1
        c = oracle.decode(T, inst.D[p], inst.R[p], inst.kM[p], inst.kR[p], inst.hM[p], inst.hR[p], em[p], er[p])[0]
        if c == INF:
            row[p, t] ^= 1
            assert applied[j] == 0
        else:
            assert applied[j] == 1
    assert (a == em).all() and (b == er).all()


def _check_records(rec, F_init, k_max):
    F = F_init
    best = F_init
    k = 1
    for i, r in enumerate(rec):
        assert r["k"] == k
        acc = r["F_local"] < F
        assert bool(r["accepted"]) == acc
        assert r["F_local"] <= r["F_shaken"]
        if acc:
            F = r["F_local"]
            k = 1
        else:
            k = 1 if k >= k_max else k + 1
        best = min(best, F)
        assert r["F_best"] == best
    return F


@pytest.mark.parametrize("k_max", [1, 3, 5])
def test_gvns_rules(k_max):
    inst = workload("plain_10x12")
    ch = oracle.Chain(inst, seed=1, chain=0, nb_list=(1, 2), k_max=k_max)
    F0 = ch.F
    rec = ch.run(60)
    assert list(rec["iter"]) == list(range(60))
    F = _check_records(rec, F0, k_max)
    assert F == ch.F == oracle.objective(inst, ch.zM, ch.zR)[0]
    assert ch.F_best == F
    price, _ = oracle.price_all(inst, ch.zM, ch.zR, 3)
    assert price.min() >= ch.F


def test_gvns_resume_equals_single_run():
    inst = draw_instance(np.random.default_rng(24), 8, 10)
    a = oracle.Chain(inst, seed=7, chain=2)
    ra = a.run(40)
    b = oracle.Chain(inst, seed=7, chain=2)
    rb = np.concatenate([b.run(15), b.run(25)])
    assert (ra == rb).all()
    assert (a.zM == b.zM).all() and (a.zR == b.zR).all() and a.k == b.k and a.F == b.F


def test_gvns_chains_differ_and_seed_determines():
    inst = workload("plain_10x12")
    r0 = oracle.Chain(inst, 1, 0, (1, 2)).run(30)
    r0b = oracle.Chain(inst, 1, 0, (1, 2)).run(30)
    r1 = oracle.Chain(inst, 1, 1, (1, 2)).run(30)
    assert (r0 == r0b).all()
    assert not (r0["F_shaken"] == r1["F_shaken"]).all()


def test_gvns_degenerate_zero_demand():
    inst = edge_instance("zero_demand", 3, 5)
    ch = oracle.Chain(inst, 1, 0)
    rec = ch.run(10)
    # with no demand every setup is removable: the first VND strips all of them
    assert ch.F == 0 and ch.zM.sum() == 0 and ch.zR.sum() == 0
    _check_records(rec, int(inst.kM.sum()) * inst.T, 5)


# ---- best-of-G (Algorithm 2: G shakes of x with the same k, each followed by the VND, the minimum kept) ----

def _numpy_draw_stream(seed, chain, it, j, g, n):
    bg = np.random.Philox(key=np.array([seed, chain], np.uint64), counter=_counter_minus_one([it, j, g, 0]))
    o0 = int(bg.random_raw(1)[0])
    return ((o0 >> 32) * n) >> 32


@pytest.mark.parametrize("g", [0, 1, 3, 15])
def test_stream_draws_match_numpy_philox(g):
    n = 2 * 100 * 52
    for it, j in ((0, 0), (7, 2), (1999, 4)):
        assert oracle.draw(5, 9, it, j, n, stream=g) == _numpy_draw_stream(5, 9, it, j, g, n)
    if g == 0:   # stream 0 is the plain chain's shake
        assert oracle.draw(5, 9, 7, 2, n) == oracle.draw(5, 9, 7, 2, n, stream=0)


def _best_of_by_hand(inst, seed, chain, nb, k_max, G, literal, iters):
    """Every iteration rebuilt from the oracle's separate steps (stream shake, VND, objective)."""
    zM = np.ones((inst.K, inst.T), np.uint8)
    zR = np.zeros((inst.K, inst.T), np.uint8)
    F, k, best, out = oracle.objective(inst, zM, zR)[0], 1, None, []
    best = F
    for it in range(iters):
        cand = []
        for g in range(G):
            a, b, _ = oracle.shake(inst, zM, zR, k, seed, chain, it, stream=g)
            Fs = oracle.objective(inst, a, b)[0]
            Fl, a2, b2, _ = oracle.vnd(inst, a, b, nb)
            cand.append((Fl, g, Fs, a2, b2))
        Fl, g, Fs, a2, b2 = min(cand, key=lambda c: (c[0], c[1]))   # lowest stream among equal values
        acc = 1 if literal else int(Fl < F)
        if acc:
            zM, zR, F = a2.reshape(inst.K, inst.T), b2.reshape(inst.K, inst.T), Fl
        best = min(best, F)
        out.append((it, k, acc, g, Fs, Fl, best))
        if not literal:
            k = 1 if acc else (1 if k >= k_max else k + 1)
    return np.array(out, dtype=oracle.RECORD_DTYPE), zM, zR


@pytest.mark.parametrize("G,literal,k_max", [(1, False, 5), (3, False, 5), (4, False, 2), (3, True, 5)])
def test_best_of_g_selects_the_minimum(G, literal, k_max):
    inst = edge_instance("uniform", 5, 9, seed=3)
    ch = oracle.BestOfChain(inst, seed=4, chain=2, nb_list=(1, 2, 4), k_max=k_max, G=G, literal=literal)
    rec = ch.run(25)
    ref, zM, zR = _best_of_by_hand(inst, 4, 2, (1, 2, 4), k_max, G, literal, 25)
    assert (rec == ref).all()
    assert (ch.zM == zM).all() and (ch.zR == zR).all()
    if literal:   # Algorithm 2 as printed: k never changes and the minimum always replaces x
        assert (rec["k"] == 1).all() and (rec["accepted"] == 1).all()
    if G > 1:
        assert (rec["winner"] > 0).any()


def test_best_of_one_is_the_plain_chain():
    inst = workload("plain_10x12")
    a = oracle.BestOfChain(inst, 1, 3, (1, 2), 5, G=1).run(50)
    b = oracle.Chain(inst, 1, 3, (1, 2)).run(50)
    assert (a == b).all()


def test_best_of_g_never_worse_than_its_first_stream():
    """At the same state, stream 0 is the plain chain's candidate, so the selected VND result is at most
    the plain one: the first iteration from the initial solution, over several chains."""
    inst = edge_instance("uniform", 6, 12, seed=8)
    for chain in range(4):
        best = oracle.BestOfChain(inst, 2, chain, (1, 2, 4), 5, G=4).run(1)[0]
        plain = oracle.Chain(inst, 2, chain).run(1)[0]
        assert best["F_local"] <= plain["F_local"]
