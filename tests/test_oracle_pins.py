"""Pins of the CPU oracle against things other than itself (CPU only).

What pins what:
  * decode: hand-worked examples (tests/golden/decode_hand.json); Wagner-Whitin DP (Wagner & Whitin 1958)
    equals the brute-force minimum over all setup patterns when there are no returns; the fixed-pattern LP of
    the Section 2 model (scipy HiGHS) equals the decode for every pattern when there are no returns and
    bounds it from below otherwise (with the same feasibility verdict); the MILP of the Section 2 model is a
    lower bound of the brute-force minimum; closed forms of lot-for-lot and single-lot plans; flow-balance
    invariants on random instances.
  * slot pricing: every slot's price against a brute-force table of all patterns, the move applied by the
    test's own integer bit operations.
  * Philox4x64-10: numpy.random.Philox and the Random123 known-answer vector.
"""
import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.optimize import Bounds, LinearConstraint, linprog, milp

import oracle
from paper_1704_05132_amd.instances import Instance, draw_instance, edge_instance, workload

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "decode_hand.json")


def _rows(bits, T):
    return np.array([(bits >> t) & 1 for t in range(T)], np.uint8)


def _one(rng, T, no_returns=False, d_hi=200):
    inst = draw_instance(rng, 1, T, d_hi=d_hi)
    if no_returns:
        inst.R[:] = 0
    return inst


def _dec(inst, zM, zR, k=0):
    return oracle.decode(inst.T, inst.D[k], inst.R[k], inst.kM[k], inst.kR[k], inst.hM[k], inst.hR[k], zM, zR)


# ----------------------------------------------------------------------------------------------------------
# Independent references: Wagner-Whitin DP, fixed-pattern LP and the MILP of the Section 2 model
# ----------------------------------------------------------------------------------------------------------
def wagner_whitin(D, kM, hM):
    """Textbook uncapacitated lot sizing DP (no returns): f[t+1] = min_j f[j] + kM + hM*sum D(tau)(tau-j)."""
    T = len(D)
    f = [0] + [None] * T
    for t in range(T):
        best = 0 if all(d == 0 for d in D[: t + 1]) else None
        for j in range(t + 1):
            if f[j] is None:
                continue
            c = f[j] + kM + hM * sum(int(D[tau]) * (tau - j) for tau in range(j, t + 1))
            best = c if best is None else min(best, c)
        f[t + 1] = best
    return f[T]


def _model(T, D, R):
    """Equality rows of the Section 2 model with variable order [xM, xR, yM, yR] (each T long)."""
    n = 4 * T
    A = np.zeros((2 * T, n))
    b = np.zeros(2 * T)
    for t in range(T):
        # yM(t) - yM(t-1) - xM(t) - xR(t) = -D(t)
        A[t, 2 * T + t] = 1
        if t > 0:
            A[t, 2 * T + t - 1] = -1
        A[t, t] = -1
        A[t, T + t] = -1
        b[t] = -D[t]
        # yR(t) - yR(t-1) + xR(t) = R(t)
        A[T + t, 3 * T + t] = 1
        if t > 0:
            A[T + t, 3 * T + t - 1] = -1
        A[T + t, T + t] = 1
        b[T + t] = R[t]
    return A, b


def lp_fixed_pattern(inst, zM, zR):
    """Optimal cost of the Section 2 model with the setup pattern fixed; None if infeasible."""
    T = inst.T
    D, R = inst.D[0].astype(float), inst.R[0].astype(float)
    big = float(D.sum() + R.sum() + 1)
    A, b = _model(T, D, R)
    c = np.concatenate([np.zeros(2 * T), np.full(T, float(inst.hM[0])), np.full(T, float(inst.hR[0]))])
    ub = np.concatenate([zM * big, zR * big, np.full(2 * T, np.inf)])
    res = linprog(c, A_eq=A, b_eq=b, bounds=list(zip(np.zeros(4 * T), ub)), method="highs")
    if res.status == 2:
        return None
    assert res.status == 0, res.message
    return res.fun + int(inst.kM[0]) * int(zM.sum()) + int(inst.kR[0]) * int(zR.sum())


def milp_optimum(inst):
    """Optimum of the Section 2 MILP (binary setups, big-M linking)."""
    T = inst.T
    D, R = inst.D[0].astype(float), inst.R[0].astype(float)
    big = float(D.sum() + R.sum() + 1)
    A, b = _model(T, D, R)
    n = 6 * T
    Aeq = np.hstack([A, np.zeros((2 * T, 2 * T))])
    link = np.zeros((2 * T, n))
    for t in range(T):
        link[t, t] = 1
        link[t, 4 * T + t] = -big
        link[T + t, T + t] = 1
        link[T + t, 5 * T + t] = -big
    c = np.concatenate([np.zeros(2 * T), np.full(T, float(inst.hM[0])), np.full(T, float(inst.hR[0])),
                        np.full(T, float(inst.kM[0])), np.full(T, float(inst.kR[0]))])
    integrality = np.concatenate([np.zeros(4 * T), np.ones(2 * T)])
    ub = np.concatenate([np.full(4 * T, np.inf), np.ones(2 * T)])
    res = milp(c, constraints=[LinearConstraint(Aeq, b, b), LinearConstraint(link, -np.inf, 0)],
               integrality=integrality, bounds=Bounds(np.zeros(n), ub))
    assert res.status == 0, res.message
    return res.fun


def brute_force(inst):
    """Decode of every (zM, zR) pattern of a one-product instance: {(bitsM, bitsR): cost}."""
    T = inst.T
    out = {}
    for bm in range(1 << T):
        zM = _rows(bm, T)
        for br in range(1 << T):
            out[(bm, br)] = _dec(inst, zM, _rows(br, T))[0]
    return out


# ----------------------------------------------------------------------------------------------------------
# decode
# ----------------------------------------------------------------------------------------------------------
def test_hand_worked_examples():
    ex = json.load(open(GOLDEN))["examples"]
    assert len(ex) >= 8
    for e in ex:
        T = len(e["D"])
        c, xM, xR, yM, yR = oracle.decode(T, np.array(e["D"]), np.array(e["R"]), e["kM"], e["kR"], e["hM"],
                                          e["hR"], np.array(e["zM"], np.uint8), np.array(e["zR"], np.uint8))
        if e["cost"] < 0:
            assert c == INF, e["name"]
            continue
        assert c == e["cost"], e["name"]
        for key, arr in (("xM", xM), ("xR", xR), ("yM", yM), ("yR", yR)):
            assert list(arr) == e[key], (e["name"], key)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("T", [1, 3, 5, 7])
def test_bruteforce_min_equals_wagner_whitin_without_returns(seed, T):
    rng = np.random.default_rng([11, seed, T])
    inst = _one(rng, T, no_returns=True)
    if seed % 4 == 0:
        inst.D[0, rng.random(T) < 0.4] = 0      # zero-demand periods, incl. leading ones
    table = brute_force(inst)
    best = min(table.values())
    assert best == wagner_whitin(inst.D[0], int(inst.kM[0]), int(inst.hM[0]))


@pytest.mark.parametrize("seed", range(4))
def test_decode_equals_lp_for_every_pattern_without_returns(seed):
    T = 4
    rng = np.random.default_rng([12, seed])
    inst = _one(rng, T, no_returns=True, d_hi=20)
    if seed == 3:
        inst.D[0, 0] = 0
    for bm, br in itertools.product(range(1 << T), repeat=2):
        zM, zR = _rows(bm, T), _rows(br, T)
        c = _dec(inst, zM, zR)[0]
        lp = lp_fixed_pattern(inst, zM, zR)
        if lp is None:
            assert c == INF, (bm, br)
        else:
            assert c == round(lp) and abs(lp - round(lp)) < 1e-6, (bm, br, c, lp)


@pytest.mark.parametrize("seed", range(4))
def test_lp_bounds_decode_with_returns(seed):
    T = 4
    rng = np.random.default_rng([13, seed])
    inst = _one(rng, T, d_hi=20)
    if seed == 2:
        inst.R[0] = rng.integers(0, 40, T)      # returns above demand
    n_feasible = 0
    for bm, br in itertools.product(range(1 << T), repeat=2):
        zM, zR = _rows(bm, T), _rows(br, T)
        c = _dec(inst, zM, zR)[0]
        lp = lp_fixed_pattern(inst, zM, zR)
        assert (lp is None) == (c == INF), (bm, br, c, lp)
        if lp is not None:
            n_feasible += 1
            assert lp <= c + 1e-6, (bm, br, c, lp)
    assert n_feasible > 0


@pytest.mark.parametrize("seed", range(6))
def test_milp_lower_bounds_bruteforce(seed):
    T = 5
    rng = np.random.default_rng([14, seed])
    inst = _one(rng, T, no_returns=(seed == 0))
    best = min(brute_force(inst).values())
    opt = milp_optimum(inst)
    assert opt <= best + 1e-6
    if seed == 0:
        assert abs(opt - best) < 1e-6   # without returns the decode reaches the MILP optimum


def test_closed_forms():
    rng = np.random.default_rng(15)
    for T in (1, 2, 12, 52, 104):
        inst = _one(rng, T)
        D, R = inst.D[0].astype(np.int64), inst.R[0].astype(np.int64)
        kM, kR, hM, hR = (int(v[0]) for v in (inst.kM, inst.kR, inst.hM, inst.hR))
        PR = np.cumsum(R)
        PD = np.cumsum(D)
        ones, zeros = np.ones(T, np.uint8), np.zeros(T, np.uint8)
        # lot-for-lot without remanufacturing: every return is held to the horizon
        assert _dec(inst, ones, zeros)[0] == T * kM + hR * int(PR.sum())
        # both setups every period with R <= D: returns used at once, nothing held
        assert (R <= D).all()
        assert _dec(inst, ones, ones)[0] == T * (kM + kR)
        # one manufacturing lot at t=0 for the whole horizon
        single = zeros.copy()
        single[0] = 1
        assert _dec(inst, single, zeros)[0] == kM + hM * int((PD[-1] - PD).sum()) + hR * int(PR.sum())


def _check_invariants(inst, zM, zR):
    T = inst.T
    c, xM, xR, yM, yR = _dec(inst, zM, zR)
    if c == INF:
        return False
    D, R = inst.D[0].astype(np.int64), inst.R[0].astype(np.int64)
    prevM = np.concatenate([[0], yM[:-1]])
    prevR = np.concatenate([[0], yR[:-1]])
    assert (yM == prevM + xM + xR - D).all()
    assert (yR == prevR + R - xR).all()
    assert (xM >= 0).all() and (xR >= 0).all() and (yM >= 0).all() and (yR >= 0).all()
    assert not (xM[zM == 0] > 0).any() and not (xR[zR == 0] > 0).any()
    assert yM[-1] == 0
    assert xM.sum() + xR.sum() == D.sum()
    assert yR[-1] == R.sum() - xR.sum()
    setup = (zM | zR).astype(bool)
    nxt = [next((u for u in range(t + 1, T) if setup[u]), T) for t in range(T)]
    shortfall = [D[t:nxt[t]].sum() - xR[t] if (setup[t] and not zM[t]) else 0 for t in range(T)]
    for t in range(T):
        if not setup[t]:
            continue
        if zR[t]:
            # remanufacture first: the lot is min(available returns, demand until the next setup)
            assert xR[t] == min(prevR[t] + R[t], D[t:nxt[t]].sum())
        if zM[t]:
            assert prevM[t] == 0                # zero inventory entering a manufacturing setup
        else:
            # stock entering a remanufacture-only setup: the shortfalls carried back through it, i.e. those
            # of the remanufacture-only setups from t up to the next manufacturing setup
            nextM = next((u for u in range(t + 1, T) if zM[u]), T)
            assert prevM[t] == sum(shortfall[t:nextM])
    cost = (int(inst.kM[0]) * int(zM.sum()) + int(inst.kR[0]) * int(zR.sum()) + int(inst.hM[0]) * int(yM.sum())
            + int(inst.hR[0]) * int(yR.sum()))
    assert c == cost
    return True


@settings(max_examples=300, deadline=None)
@given(T=st.integers(1, 40), seed=st.integers(0, 2**31), dens=st.floats(0.05, 0.95),
       kind=st.sampled_from(["uniform", "no_returns", "returns_eq_demand", "big_returns", "sparse",
                             "zero_demand"]))
def test_decode_invariants(T, seed, dens, kind):
    inst = edge_instance(kind, 1, T, seed)
    rng = np.random.default_rng(seed)
    zM = (rng.random(T) < dens).astype(np.uint8)
    zR = (rng.random(T) < dens).astype(np.uint8)
    _check_invariants(inst, zM, zR)
    zM[0] = 1
    assert _check_invariants(inst, zM, zR)    # a manufacturing setup in period 0 is always feasible


# ----------------------------------------------------------------------------------------------------------
# slot pricing and argmin
# ----------------------------------------------------------------------------------------------------------
def _moved(bm, br, T, l):
    """The test's own move application on integer bit rows: (bm', br') or None for a non-move."""
    if l < T:
        return bm ^ (1 << l), br
    if l < 2 * T:
        return bm, br ^ (1 << (l - T))
    t = l - 2 * T if l < 3 * T else l - 3 * T
    z = bm if l < 3 * T else br
    if t >= T - 1 or ((z >> t) & 1) == ((z >> (t + 1)) & 1):
        return None
    z ^= (1 << t) | (1 << (t + 1))
    return (z, br) if l < 3 * T else (bm, z)


@pytest.mark.parametrize("T", [1, 2, 4, 5])
@pytest.mark.parametrize("seed", range(3))
def test_prices_against_bruteforce_table(T, seed):
    rng = np.random.default_rng([16, T, seed])
    inst = _one(rng, T, d_hi=50)
    table = brute_force(inst)
    feasible = [p for p, c in table.items() if c != INF]
    picks = [feasible[i] for i in rng.choice(len(feasible), size=min(25, len(feasible)), replace=False)]
    for bm, br in picks:
        F = table[(bm, br)]
        for mask in (1, 2, 4, 7, 3):
            price, n = oracle.price_all(inst, _rows(bm, T)[None], _rows(br, T)[None], mask)
            n_expect = 0
            for l in range(4 * T):
                nb = 1 if l < T else (2 if l < 2 * T else 4)
                mv = _moved(bm, br, T, l)
                if not (nb & mask) or mv is None:
                    assert price[l] == INF
                    continue
                n_expect += 1
                c = table[mv]
                assert price[l] == (INF if c == INF else c), (bm, br, l)
            assert n == n_expect
            v, s = oracle.argmin(price)
            finite = [(p, i) for i, p in enumerate(price) if p != INF]
            assert (v, s) == (min(finite) if finite else (INF, -1))


def test_argmin_lowest_slot_on_ties():
    p = np.array([INF, 5, 3, 3, 9, 3], np.int64)
    assert oracle.argmin(p) == (3, 2)
    assert oracle.argmin(np.full(4, INF, np.int64)) == (INF, -1)


def test_prices_multi_product_are_relative_to_F():
    inst = workload("plain_10x12")
    rng = np.random.default_rng(17)
    zM = (rng.random((inst.K, inst.T)) < 0.5).astype(np.uint8)
    zM[:, 0] = 1
    zR = (rng.random((inst.K, inst.T)) < 0.3).astype(np.uint8)
    F, cost = oracle.objective(inst, zM, zR)
    price, _ = oracle.price_all(inst, zM, zR, 7)
    T = inst.T
    for k in range(inst.K):
        sub = inst.product(k)
        pk, _ = oracle.price_all(sub, zM[k:k + 1], zR[k:k + 1], 7)
        blk = price[4 * T * k: 4 * T * (k + 1)]
        fin = pk != INF
        assert ((blk != INF) == fin).all()
        assert (blk[fin] == pk[fin] - cost[k] + F).all()   # F' = F - cost_k + cost_k(moved)


# ----------------------------------------------------------------------------------------------------------
# Philox4x64-10
# ----------------------------------------------------------------------------------------------------------
def test_philox_known_answer():
    kat = json.load(open(GOLDEN))["philox4x64_10_known_answer"]
    out = oracle.philox4x64_10([int(x, 16) for x in kat["key"]], [int(x, 16) for x in kat["counter"]])
    assert [hex(int(x)) for x in out] == kat["out"]


@pytest.mark.parametrize("key0,key1,c0,c1", [(1, 0, 0, 0), (2, 63, 1999, 4), (3, 32767, 5, 0),
                                              (2**63 + 5, 2**40, 2**33, 7)])
def test_philox_matches_numpy(key0, key1, c0, c1):
    key = np.array([key0, key1], np.uint64)
    ctr = np.array([c0, c1, 0, 0], np.uint64)
    # numpy's Philox increments its counter before producing a block
    ref = np.random.Philox(key=key, counter=ctr).random_raw(4)
    nxt = ctr.copy()
    nxt[0] += np.uint64(1)
    assert (oracle.philox4x64_10(key, nxt) == ref).all()


# ---- unit costs p_M, p_R (the parameters Algorithm 1's signature carries) ----

def _forward_remanufactured(T, D, R, zM, zR):
    """Total remanufactured quantity by the forward recurrence of the decode (capacity closed at a
    manufacturing setup, reopened to all returns so far at a remanufacturing setup), written out here
    independently of the oracle's look-ahead decode."""
    lim = XR = PR = 0
    for t in range(T):
        PR += int(R[t])
        if zM[t]:
            lim = XR
        if zR[t]:
            lim = PR
        XR = min(XR + int(D[t]), lim)
    return XR


@pytest.mark.parametrize("seed", range(6))
def test_unit_costs_of_the_items_made(seed):
    rng = np.random.default_rng(1000 + seed)
    inst = draw_instance(rng, 3, 11)
    checked = 0
    for _ in range(60):
        zM = (rng.random((inst.K, inst.T)) < 0.4).astype(np.uint8)
        zR = (rng.random((inst.K, inst.T)) < 0.4).astype(np.uint8)
        zM[:, 0] |= rng.random(inst.K) < 0.8
        for k in range(inst.K):
            args = (inst.T, inst.D[k], inst.R[k], inst.kM[k], inst.kR[k], inst.hM[k], inst.hR[k], zM[k], zR[k])
            c0 = oracle.decode(*args)[0]
            if c0 == INF:
                assert oracle.decode(*args, pM=5, pR=9)[0] == INF
                continue
            sD = int(inst.D[k].sum())
            p = int(rng.integers(1, 60))
            assert oracle.decode(*args, pM=p, pR=p)[0] == c0 + p * sD   # every demanded unit is made once
            pM, pR = (int(v) for v in rng.integers(0, 60, 2))
            X = _forward_remanufactured(inst.T, inst.D[k], inst.R[k], zM[k], zR[k])
            assert oracle.decode(*args, pM=pM, pR=pR)[0] == c0 + pM * (sD - X) + pR * X
            checked += 1
    assert checked > 20


def test_unit_costs_without_returns_shift_the_optimum():
    """Without returns nothing is remanufactured: p_M adds p_M * sum(D) to every feasible pattern, so the
    brute-force optimum moves by exactly that and p_R does not matter."""
    rng = np.random.default_rng(77)
    inst = draw_instance(rng, 1, 6)
    inst.R[:] = 0
    sD = int(inst.D[0].sum())
    best0 = best1 = INF
    for bits in range(1 << (2 * inst.T)):
        zM = _rows(bits, inst.T)
        zR = _rows(bits >> inst.T, inst.T)
        args = (inst.T, inst.D[0], inst.R[0], inst.kM[0], inst.kR[0], inst.hM[0], inst.hR[0], zM, zR)
        best0 = min(best0, oracle.decode(*args)[0])
        best1 = min(best1, oracle.decode(*args, pM=13, pR=999)[0])
    assert best1 == best0 + 13 * sD


def test_unit_costs_in_the_search():
    """The instance's unit costs reach every part of the search: the objective of the final solution, the
    VND's local optimum and the GVNS records use them."""
    inst = draw_instance(np.random.default_rng(5), 6, 10)
    inst.pM = np.full(inst.K, 40, np.int32)
    inst.pR = np.full(inst.K, 3, np.int32)   # cheap remanufacturing: the optimum keeps more zR setups
    ch = oracle.Chain(inst, 1, 0)
    rec = ch.run(30)
    assert ch.F == oracle.objective(inst, ch.zM, ch.zR)[0]
    assert rec["F_best"][-1] == ch.F_best
    price, _ = oracle.price_all(inst, ch.zM, ch.zR, 7)
    assert price.min() >= ch.F
    plain = draw_instance(np.random.default_rng(5), 6, 10)
    assert oracle.objective(inst, ch.zM, ch.zR)[0] != oracle.objective(plain, ch.zM, ch.zR)[0]


# ----------------------------------------------------------------------------------------------------------
# The strict reading of a remanufacture-only shortfall (R5-alt)
# ----------------------------------------------------------------------------------------------------------
GOLDEN_STRICT = os.path.join(os.path.dirname(__file__), "golden", "decode_strict_hand.json")


def test_strict_hand_worked_examples():
    with open(GOLDEN_STRICT) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        T = len(e["D"])
        args = (T, np.array(e["D"], np.int32), np.array(e["R"], np.int32), e["kM"], e["kR"], e["hM"], e["hR"],
                np.array(e["zM"], np.uint8), np.array(e["zR"], np.uint8))
        c_strict = oracle.decode(*args, strict=True)[0]
        c_carry = oracle.decode(*args)[0]
        assert (c_strict if c_strict != INF else -1) == e["cost"], e["name"]
        assert (c_carry if c_carry != INF else -1) == e["carry_back_cost"], e["name"]


def _carried(inst, zM, zR):
    """Whether the carry-back decode moved a shortfall: stock held into a setup period (the look-ahead decode
    ends every setup interval with empty serviceable stock unless a later shortfall was carried back)."""
    c, xM, xR, yM, yR = _dec(inst, zM, zR)
    if c == INF:
        return None
    setups = np.nonzero(np.asarray(zM) | np.asarray(zR))[0]
    return any(t >= 1 and yM[t - 1] > 0 for t in setups)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("T", [1, 3, 5])
def test_strict_is_carry_back_without_a_carried_shortfall(seed, T):
    """Every pattern: the strict decode is feasible exactly where the carry-back decode is feasible and moved
    no shortfall, and then both give the same lots and cost."""
    rng = np.random.default_rng([71, seed, T])
    inst = _one(rng, T)
    if seed % 3 == 1:
        inst.R[0] = rng.integers(0, 400, T)   # returns above demand too
    n_infeasible = 0
    for bm in range(1 << T):
        for br in range(1 << T):
            zM, zR = _rows(bm, T), _rows(br, T)
            carried = _carried(inst, zM, zR)
            st = oracle.decode(inst.T, inst.D[0], inst.R[0], inst.kM[0], inst.kR[0], inst.hM[0], inst.hR[0], zM, zR,
                               strict=True)
            if carried is None or carried:
                assert st[0] == INF, (bm, br)
                n_infeasible += carried is True
            else:
                cb = _dec(inst, zM, zR)
                assert st[0] == cb[0], (bm, br)
                for a, b in zip(st[1:], cb[1:]):
                    assert (a == b).all()
    if T >= 3:
        assert n_infeasible > 0


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("T", [2, 4, 6])
def test_strict_bruteforce_min_equals_wagner_whitin_without_returns(seed, T):
    """Without returns a remanufacture-only interval with demand is infeasible under the strict reading, so
    its brute-force optimum is the textbook lot-sizing optimum."""
    rng = np.random.default_rng([72, seed, T])
    inst = _one(rng, T, no_returns=True)
    inst.strict = True
    best = min(oracle.objective(inst, _rows(bm, T)[None, :], _rows(br, T)[None, :])[0]
               for bm in range(1 << T) for br in range(1 << T))
    assert best == wagner_whitin(inst.D[0], int(inst.kM[0]), int(inst.hM[0]))


def test_strict_search_states_are_strict_feasible():
    """The oracle's search under the strict reading moves only between strictly feasible patterns, and every
    reported objective is the strict objective of the state."""
    inst = edge_instance("uniform", 6, 14, seed=3)
    inst.strict = True
    ch = oracle.Chain(inst, 5, 0)
    rec = ch.run(25)
    F = oracle.objective(inst, ch.zM, ch.zR)[0]
    assert F == ch.F != INF and (rec["F_local"] <= rec["F_shaken"]).all()
    price, _ = oracle.price_all(inst, ch.zM, ch.zR, 7)
    assert price.min() >= F
    # the same state under the carry-back reading costs the same (it moves no shortfall)
    inst2 = edge_instance("uniform", 6, 14, seed=3)
    assert oracle.objective(inst2, ch.zM, ch.zR)[0] == F


# ----------------------------------------------------------------------------------------------------------
# Disposal of returns no lot needs (R29)
# ----------------------------------------------------------------------------------------------------------
GOLDEN_DISPOSE = os.path.join(os.path.dirname(__file__), "golden", "decode_dispose_hand.json")


def test_dispose_hand_worked_examples():
    with open(GOLDEN_DISPOSE) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        T = len(e["D"])
        args = (T, np.array(e["D"], np.int32), np.array(e["R"], np.int32), e["kM"], e["kR"], e["hM"], e["hR"],
                np.array(e["zM"], np.uint8), np.array(e["zR"], np.uint8))
        assert oracle.decode(*args, dispose=True)[0] == e["cost"], e["name"]
        assert oracle.decode(*args)[0] == e["no_disposal_cost"], e["name"]


def lp_kept_recoverable(R, xR):
    """Least total recoverable stock with the lots fixed and free disposal: min sum y(t) subject to
    y(t) = y(t-1) + R(t) - xR(t) - w(t), y >= 0, w >= 0 (variables [y, w]); scipy HiGHS."""
    T = len(R)
    A = np.zeros((T, 2 * T))
    b = np.zeros(T)
    for t in range(T):
        A[t, t] = 1
        if t > 0:
            A[t, t - 1] = -1
        A[t, T + t] = 1
        b[t] = R[t] - xR[t]
    r = linprog(np.r_[np.ones(T), np.zeros(T)], A_eq=A, b_eq=b, bounds=[(0, None)] * (2 * T), method="highs")
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("T", [2, 4, 5])
@pytest.mark.parametrize("strict", [False, True])
def test_dispose_holding_is_the_disposal_lp_optimum(seed, T, strict):
    """Every pattern: the lots do not change, and the recoverable holding charged is hR times the least
    recoverable stock any disposal plan keeps for those lots (an LP over the disposals)."""
    rng = np.random.default_rng([73, seed, T])
    inst = _one(rng, T)
    if seed % 2:
        inst.R[0] = rng.integers(0, 300, T)
    k = 0
    n_saved = 0
    for bm in range(1 << T):
        for br in range(1 << T):
            zM, zR = _rows(bm, T), _rows(br, T)
            a = (inst.T, inst.D[k], inst.R[k], inst.kM[k], inst.kR[k], inst.hM[k], inst.hR[k], zM, zR)
            c0, xM, xR, yM, yR = oracle.decode(*a, strict=strict)
            c1, xM1, xR1, yM1, yR1 = oracle.decode(*a, strict=strict, dispose=True)
            if c0 == INF:
                assert c1 == INF
                continue
            assert (xM1 == xM).all() and (xR1 == xR).all() and (yM1 == yM).all()
            kept = lp_kept_recoverable(inst.R[k], xR)
            expect = c0 - int(inst.hR[k]) * int(yR.sum()) + int(inst.hR[k]) * int(round(kept))
            assert c1 == expect, (bm, br)
            n_saved += c1 < c0
    assert n_saved > 0


def test_dispose_without_returns_changes_nothing():
    rng = np.random.default_rng(74)
    for T in (1, 3, 6):
        inst = _one(rng, T, no_returns=True)
        for bm in range(1 << T):
            for br in range(1 << T):
                zM, zR = _rows(bm, T), _rows(br, T)
                a = (inst.T, inst.D[0], inst.R[0], inst.kM[0], inst.kR[0], inst.hM[0], inst.hR[0], zM, zR)
                assert oracle.decode(*a, dispose=True)[0] == oracle.decode(*a)[0]


def test_dispose_in_the_search():
    """The oracle's search with disposal: objective of every state recomputed, local optimality, and the
    disposal objective never above the no-disposal one of the same state."""
    inst = edge_instance("big_returns", 5, 12, seed=6)
    inst.dispose = True
    ch = oracle.Chain(inst, 3, 1)
    ch.run(20)
    F = oracle.objective(inst, ch.zM, ch.zR)[0]
    assert F == ch.F
    price, _ = oracle.price_all(inst, ch.zM, ch.zR, 7)
    assert price.min() >= F
    plain = edge_instance("big_returns", 5, 12, seed=6)
    assert oracle.objective(plain, ch.zM, ch.zR)[0] >= F
