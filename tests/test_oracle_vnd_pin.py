"""Pins of the oracle's VND (Algorithm 1) move selection, CPU only.

The VND here is written in the test from the algorithm's statement and the neighbourhood definitions,
over brute-force tables: the decode cost of every one of the 2^(2T) setup patterns of each product (the
decode is pinned on its own in test_oracle_pins.py).  Moves are the test's own bit operations on a pattern
integer (zM in bits 0..T-1, zR in bits T..2T-1).  For each pass, neighbourhoods are taken in list order and,
for each of them, every product's lowest (price, slot) move is applied only if it strictly lowers F; a pass
never goes back to the first neighbourhood; passes repeat until one applies nothing.  The oracle's VND must
apply the same moves in the same order and end on the same patterns.

A hand-worked example (tests/golden/vnd_hand.json) anchors the rule independently of any code, and the
comparison is shown to catch plausible mistakes: copies of the oracle source with a planted mistake
(first improvement, a return to the first neighbourhood after an improvement, ties to the higher slot,
products before neighbourhoods) are compiled on the CPU and must fail it.
"""
import ctypes
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1704_05132_amd.instances import Instance, draw_instance

INF = oracle.INF
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "vnd_hand.json")


# ---------------------------------------------------------------------------------------------------
# the test's own VND over cost tables
# ---------------------------------------------------------------------------------------------------
def _bits(v, T):
    return np.array([(v >> t) & 1 for t in range(T)], np.uint8)


def cost_table(inst, k):
    """Decode cost of every pattern of product k: index zM | zR << T."""
    T = inst.T
    pM, pR = inst.unit_costs()
    tab = np.empty(1 << (2 * T), np.int64)
    for v in range(1 << (2 * T)):
        tab[v] = oracle.decode(T, inst.D[k], inst.R[k], inst.kM[k], inst.kR[k], inst.hM[k], inst.hR[k],
                               _bits(v, T), _bits(v >> T, T), pM[k], pR[k])[0]
    return tab


def moves(v, T, nb):
    """(slot, new pattern) of every move of neighbourhood nb from pattern v, slots in increasing order."""
    out = []
    if nb == 1:
        out = [(t, v ^ (1 << t)) for t in range(T)]
    elif nb == 2:
        out = [(T + t, v ^ (1 << (T + t))) for t in range(T)]
    elif nb == 4:
        for row in (0, 1):             # shift a zM setup, then a zR setup, by one period
            for t in range(T - 1):
                a, b = row * T + t, row * T + t + 1
                if ((v >> a) & 1) != ((v >> b) & 1):
                    out.append(((2 + row) * T + t, v ^ (1 << a) ^ (1 << b)))
    return out


def reference_vnd(tabs, T, pats, nb_list):
    pats = list(pats)
    cost = [int(tabs[k][pats[k]]) for k in range(len(pats))]
    F = sum(cost)
    trace, p = [], 0
    while True:
        improved = False
        for nb in nb_list:
            for k in range(len(pats)):
                best = None
                for slot, nv in moves(pats[k], T, nb):
                    c = int(tabs[k][nv])
                    if c == INF:
                        continue
                    cand = (F - cost[k] + c, slot, nv, c)
                    if best is None or cand[:2] < best[:2]:
                        best = cand
                if best is not None and best[0] < F:
                    F, pats[k], cost[k] = best[0], best[2], best[3]
                    trace.append((p, nb, k, best[1], F))
                    improved = True
        p += 1
        if not improved:
            return F, pats, trace


def pattern_of(zM_row, zR_row, T):
    return int(sum(int(zM_row[t]) << t for t in range(T)) + sum(int(zR_row[t]) << (T + t) for t in range(T)))


def feasible_start(rng, tabs, T):
    pats = []
    for tab in tabs:
        while True:
            v = int(rng.integers(0, 1 << (2 * T)))
            if tab[v] != INF:
                pats.append(v)
                break
    return pats


def _cases():
    """Instances of 1-3 products, T 3..6, among them constant demands (ties between moves) and returns."""
    cases = []
    for seed in range(10):
        rng = np.random.default_rng([71, seed])
        T = 3 + seed % 4 if seed < 8 else 6
        K = 1 + seed % 3
        inst = draw_instance(rng, K, T, d_hi=40)
        if seed % 2 == 1:                         # constant demand and costs: many equal prices
            inst.D[:] = 10
            inst.R[:] = (inst.R > 0) * 4
        cases.append((seed, inst))
    return cases


CASES = _cases()
_TABS = {}


def _tabs(seed, inst):
    if seed not in _TABS:
        _TABS[seed] = [cost_table(inst, k) for k in range(inst.K)]
    return _TABS[seed]


def _compare(vnd_fn, seed, inst, nb_list, starts=3):
    """True when vnd_fn agrees with the reference move by move from `starts` random feasible starts."""
    tabs = _tabs(seed, inst)
    T = inst.T
    rng = np.random.default_rng([72, seed, len(nb_list)])
    for _ in range(starts):
        pats = feasible_start(rng, tabs, T)
        zM = np.array([_bits(v, T) for v in pats])
        zR = np.array([_bits(v >> T, T) for v in pats])
        F_ref, pats_ref, tr_ref = reference_vnd(tabs, T, pats, nb_list)
        F, a, b, _, tr = vnd_fn(inst, zM, zR, nb_list)
        got = [pattern_of(a[k], b[k], T) for k in range(inst.K)]
        if F != F_ref or got != pats_ref or [tuple(int(x) for x in r) for r in tr] != tr_ref:
            return False
    return True


@pytest.mark.parametrize("nb_list", [(1, 2, 4), (4, 2, 1), (1, 2), (2, 4)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_vnd_moves_equal_brute_force_reference(case, nb_list):
    seed, inst = CASES[case]
    assert _compare(lambda *a: oracle.vnd(*a, trace=True), seed, inst, nb_list)


def test_vnd_hand_worked_example():
    with open(GOLDEN) as f:
        g = json.load(f)
    T = g["T"]
    P = g["products"]
    arr = lambda key: np.array([p[key] for p in P], np.int32)
    inst = Instance(len(P), T, arr("D"), arr("R"), arr("kM"), arr("kR"), arr("hM"), arr("hR"), "vnd_hand")
    zM = np.array([p["zM"] for p in P], np.uint8)
    zR = np.array([p["zR"] for p in P], np.uint8)
    F0, cost0 = oracle.objective(inst, zM, zR)
    assert F0 == g["F0"] and list(cost0) == [p["cost0"] for p in P]
    F, a, b, _, tr = oracle.vnd(inst, zM, zR, tuple(g["nb_list"]), trace=True)
    assert F == g["F"]
    assert tr.tolist() == g["moves"]
    assert a.tolist() == g["final_zM"] and b.tolist() == g["final_zR"]
    # the test's own VND agrees with the hand-worked moves as well
    tabs = [cost_table(inst, k) for k in range(inst.K)]
    Fr, _, trr = reference_vnd(tabs, T, [pattern_of(zM[k], zR[k], T) for k in range(inst.K)], g["nb_list"])
    assert Fr == g["F"] and [list(r) for r in trr] == g["moves"]


# ---------------------------------------------------------------------------------------------------
# planted mistakes: each mutated copy of the oracle must fail the comparison above
# ---------------------------------------------------------------------------------------------------
BEST = "if (p < best_price) { best_price = p; best_l = l; }"
MUTATIONS = {
    "first_improvement": [(BEST, "if (p < best_price) { best_price = p; best_l = l; if (p < F) break; }")],
    "ties_to_higher_slot": [(BEST, "if (p <= best_price) { best_price = p; best_l = l; }")],
    "reset_to_first_neighbourhood": [
        ("int64_t pass = 0, n_moves = 0;", "int64_t pass = 0, n_moves = 0; int moved_q = 0;"),
        ("                    ++n_moves;\n                }\n            }\n",
         "                    ++n_moves;\n                    moved_q = 1;\n                }\n            }\n"
         "            if (moved_q) { moved_q = 0; q = -1; }\n"),
    ],
    "products_before_neighbourhoods": [
        ("for (int q = 0; q < n_nb; ++q) {\n            for (int k = 0; k < K; ++k) {",
         "for (int k = 0; k < K; ++k) {\n            for (int q = 0; q < n_nb; ++q) {"),
    ],
}


def _mutant(name, tmp):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "vns_oracle.c")).read()
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    c = os.path.join(tmp, f"{name}.c")
    so = os.path.join(tmp, f"{name}.so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", c, "-o", so], check=True)
    L = ctypes.CDLL(so)
    base = oracle.lib()
    L.orc_vnd_trace.restype = base.orc_vnd_trace.restype
    L.orc_vnd_trace.argtypes = base.orc_vnd_trace.argtypes

    def vnd_fn(inst, zM, zR, nb_list):
        a = np.ascontiguousarray(zM, np.uint8).copy()
        b = np.ascontiguousarray(zR, np.uint8).copy()
        nb = np.ascontiguousarray(nb_list, np.int32)
        cap = 4096
        rec = np.zeros(5 * cap, np.int64)
        n, ev = ctypes.c_int64(0), ctypes.c_int64(0)
        F = L.orc_vnd_trace(inst.K, inst.T, *inst.arrays(), *inst.unit_costs(), a, b, nb, len(nb),
                            ctypes.byref(ev), rec, cap, ctypes.byref(n))
        return int(F), a, b, int(ev.value), rec[:5 * min(n.value, cap)].reshape(-1, 5)

    return vnd_fn


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        fn = _mutant(name, tmp)
        caught = not all(_compare(fn, seed, inst, nb_list) for seed, inst in CASES
                         for nb_list in ((1, 2, 4), (4, 2, 1)))
    assert caught, name
