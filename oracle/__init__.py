"""CPU oracle for the lot-sizing VNS — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.  The product
library never calls it and has no fallback to it.  It wraps the plain C in `vns_oracle.c` (built into
`liboracle.so` by `oracle/build.py`) with numpy marshalling; it shares no code with the HIP path.

Parity status per function (what pins it, see tests/test_oracle_pins.py):
  decode         brute force vs Wagner-Whitin DP and per-pattern LP(z) equality when R = 0; LP(z) <= decode
                 and MILP <= min decode when R > 0; closed forms; hand-worked golden examples; flow-balance
                 invariants on random instances.
  decode, strict (a remanufacture-only shortfall is infeasible): equal to the carry-back decode wherever the
                 carry-back decode moved no shortfall, infeasible exactly where it did (every pattern of small
                 instances); hand-worked golden examples.
  decode, disposal (unneeded returns disposed of): the recoverable holding equals the optimum of the LP that
                 keeps the decode's lots and chooses the disposals (scipy HiGHS), for every pattern of small
                 instances; unchanged without returns; hand-worked golden examples.
  price_all      brute-force table of all 2^(2T) patterns (K = 1, T <= 6): every slot's price.
  vnd            move by move against a VND written in the tests over brute-force cost tables of every
                 pattern (the per-product best move of each neighbourhood in list order, applied only when
                 strictly better, lowest slot on ties, no reset within a pass); a hand-worked example
                 (tests/golden/vnd_hand.json); local optimality, monotone objective, per-product
                 independence.
  philox         numpy.random.Philox (the library's Philox4x64-10).
  shake          slots derived from numpy.random.Philox outputs; feasibility of every applied flip.
  gvns           acceptance rule, k schedule, best tracking, resume equivalence, objective recomputation.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

INF = np.iinfo(np.int64).max
_HERE = Path(__file__).resolve().parent
_LIB = None

RECORD_DTYPE = np.dtype([("iter", np.int32), ("k", np.int32), ("accepted", np.int32), ("winner", np.int32),
                         ("F_shaken", np.int64), ("F_local", np.int64), ("F_best", np.int64)])

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_recp = np.ctypeslib.ndpointer(dtype=RECORD_DTYPE, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _LIB
    if _LIB is None:
        path = _HERE / "liboracle.so"
        if not path.exists():
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(str(path))
        c = ctypes
        inst = [_i32p] * 8   # D, R, kM, kR, hM, hR, pM, pR
        L.orc_set_strict.restype = None
        L.orc_set_strict.argtypes = [c.c_int]
        L.orc_set_dispose.restype = None
        L.orc_set_dispose.argtypes = [c.c_int]
        L.orc_decode.restype = c.c_int64
        L.orc_decode.argtypes = [c.c_int, _i32p, _i32p] + [c.c_int64] * 6 + [_u8p, _u8p, _i64p, _i64p, _i64p, _i64p]
        L.orc_objective.restype = c.c_int64
        L.orc_objective.argtypes = [c.c_int, c.c_int] + inst + [_u8p, _u8p, _i64p]
        L.orc_apply_slot.restype = c.c_int
        L.orc_apply_slot.argtypes = [c.c_int, _u8p, _u8p, c.c_int]
        L.orc_price_all.restype = c.c_int64
        L.orc_price_all.argtypes = [c.c_int, c.c_int] + inst + [_u8p, _u8p, c.c_uint32, _i64p]
        L.orc_argmin.restype = c.c_int64
        L.orc_argmin.argtypes = [c.c_int64, _i64p, c.POINTER(c.c_int64)]
        L.orc_vnd.restype = c.c_int64
        L.orc_vnd.argtypes = [c.c_int, c.c_int] + inst + [_u8p, _u8p, _i32p, c.c_int, c.POINTER(c.c_int64)]
        L.orc_vnd_trace.restype = c.c_int64
        L.orc_vnd_trace.argtypes = ([c.c_int, c.c_int] + inst + [_u8p, _u8p, _i32p, c.c_int, c.POINTER(c.c_int64),
                                                                  _i64p, c.c_int64, c.POINTER(c.c_int64)])
        L.orc_philox4x64_10.restype = None
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_draw.restype = c.c_int64
        L.orc_draw.argtypes = [c.c_uint64] * 5
        L.orc_shake.restype = c.c_int
        L.orc_shake.argtypes = [c.c_int, c.c_int] + inst + [_u8p, _u8p, c.c_int, c.c_uint64, c.c_uint64,
                                                            c.c_uint64, _i32p]
        L.orc_gvns.restype = c.c_int64
        L.orc_gvns.argtypes = ([c.c_int, c.c_int] + inst +
                               [_u8p, _u8p, _i32p, c.c_int, c.c_int, c.c_uint64, c.c_uint64, c.c_int64,
                                c.c_int64, c.POINTER(c.c_int32), c.POINTER(c.c_int64), _recp,
                                c.POINTER(c.c_int64)])
        L.orc_draw_stream.restype = c.c_int64
        L.orc_draw_stream.argtypes = [c.c_uint64] * 6
        L.orc_shake_stream.restype = c.c_int
        L.orc_shake_stream.argtypes = [c.c_int, c.c_int] + inst + [_u8p, _u8p, c.c_int, c.c_uint64, c.c_uint64,
                                                                   c.c_uint64, c.c_uint64, _i32p]
        L.orc_gvns_best_of.restype = c.c_int64
        L.orc_gvns_best_of.argtypes = ([c.c_int, c.c_int] + inst +
                                       [_u8p, _u8p, _i32p, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                        c.c_uint64, c.c_int64, c.c_int64, c.POINTER(c.c_int32),
                                        c.POINTER(c.c_int64), _recp, c.POINTER(c.c_int64)])
        _LIB = L
    return _LIB


def _inst(inst):
    """The instance's arrays for a call, with its decode readings (carry-back or strict; disposal or not) put
    in force."""
    lib().orc_set_strict(1 if getattr(inst, "strict", False) else 0)
    lib().orc_set_dispose(1 if getattr(inst, "dispose", False) else 0)
    return inst.arrays() + inst.unit_costs()


def _rows(z, K, T):
    a = np.ascontiguousarray(np.asarray(z, dtype=np.uint8).reshape(K, T))
    return a


def decode(T, D, R, kM, kR, hM, hR, zM, zR, pM=0, pR=0, strict=False, dispose=False):
    """Decode one product: returns (cost, xM, xR, yM, yR); cost is INF when infeasible.  pM, pR: unit costs of
    a manufactured and a remanufactured item; strict: a remanufacture-only shortfall is infeasible instead of
    carried back; dispose: returns no lot needs are disposed of (recoverable holding only on the kept stock;
    yR is still the stock without disposal)."""
    xM, xR, yM, yR = (np.zeros(T, np.int64) for _ in range(4))
    lib().orc_set_strict(1 if strict else 0)
    lib().orc_set_dispose(1 if dispose else 0)
    c = lib().orc_decode(int(T), np.ascontiguousarray(D, np.int32), np.ascontiguousarray(R, np.int32),
                         int(kM), int(kR), int(hM), int(hR), int(pM), int(pR), np.ascontiguousarray(zM, np.uint8),
                         np.ascontiguousarray(zR, np.uint8), xM, xR, yM, yR)
    return int(c), xM, xR, yM, yR


def objective(inst, zM, zR):
    """(F, cost per product) of a solution given as [K, T] bit rows."""
    cost = np.zeros(inst.K, np.int64)
    F = lib().orc_objective(inst.K, inst.T, *_inst(inst), _rows(zM, inst.K, inst.T),
                            _rows(zR, inst.K, inst.T), cost)
    return int(F), cost


def apply_slot(T, zM_row, zR_row, l):
    """Apply local slot l to copies of one product's rows; returns (valid, zM, zR)."""
    a = np.ascontiguousarray(zM_row, np.uint8).copy()
    b = np.ascontiguousarray(zR_row, np.uint8).copy()
    ok = lib().orc_apply_slot(int(T), a, b, int(l))
    return bool(ok), a, b


def price_all(inst, zM, zR, nb_mask=7):
    """Prices of all 4KT slots (INF where not a priced move) and the number of move-evaluations."""
    price = np.zeros(4 * inst.K * inst.T, np.int64)
    n = lib().orc_price_all(inst.K, inst.T, *_inst(inst), _rows(zM, inst.K, inst.T),
                            _rows(zR, inst.K, inst.T), int(nb_mask), price)
    return price, int(n)


def argmin(price):
    """Lexicographic (price, slot) minimum; (INF, -1) when nothing is priced."""
    p = np.ascontiguousarray(price, np.int64)
    s = ctypes.c_int64(0)
    v = lib().orc_argmin(len(p), p, ctypes.byref(s))
    return int(v), int(s.value)


def vnd(inst, zM, zR, nb_list=(1, 2, 4), trace=False):
    """VND (Algorithm 1) from the given solution; returns (F, zM, zR, move-evaluations), and with `trace`
    also the applied moves as an int64 array of rows (pass, neighbourhood id, product, local slot, F after)."""
    a = _rows(zM, inst.K, inst.T).copy()
    b = _rows(zR, inst.K, inst.T).copy()
    ev = ctypes.c_int64(0)
    nb = np.ascontiguousarray(nb_list, np.int32)
    if not trace:
        F = lib().orc_vnd(inst.K, inst.T, *_inst(inst), a, b, nb, len(nb), ctypes.byref(ev))
        return int(F), a, b, int(ev.value)
    cap = 1 << 12
    while True:
        rec = np.zeros(5 * cap, np.int64)
        n = ctypes.c_int64(0)
        a = _rows(zM, inst.K, inst.T).copy()
        b = _rows(zR, inst.K, inst.T).copy()
        ev = ctypes.c_int64(0)
        F = lib().orc_vnd_trace(inst.K, inst.T, *_inst(inst), a, b, nb, len(nb), ctypes.byref(ev), rec, cap,
                                ctypes.byref(n))
        if n.value <= cap:
            return int(F), a, b, int(ev.value), rec[:5 * n.value].reshape(-1, 5)
        cap = int(n.value)


def philox4x64_10(key, ctr):
    """One Philox4x64-10 block for key (2 words) and counter (4 words)."""
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(np.asarray(key, np.uint64), np.asarray(ctr, np.uint64), out)
    return out


def draw(seed, chain, it, j, n, stream=0):
    """Draw j of iteration it of random stream `stream` (Philox counter (it, j, stream, 0)), in [0, n)."""
    if stream:
        return int(lib().orc_draw_stream(seed, chain, it, j, stream, n))
    return int(lib().orc_draw(seed, chain, it, j, n))


def shake(inst, zM, zR, k, seed, chain, it, stream=0):
    """Shake(x, k) with random stream `stream`: returns (zM, zR, applied flags per draw)."""
    a = _rows(zM, inst.K, inst.T).copy()
    b = _rows(zR, inst.K, inst.T).copy()
    applied = np.zeros(max(k, 1), np.int32)
    if stream:
        lib().orc_shake_stream(inst.K, inst.T, *_inst(inst), a, b, int(k), seed, chain, it, stream, applied)
    else:
        lib().orc_shake(inst.K, inst.T, *_inst(inst), a, b, int(k), seed, chain, it, applied)
    return a, b, applied[:k]


class Chain:
    """One GVNS chain of the oracle: state (x, k, best) and resumable runs."""

    def __init__(self, inst, seed, chain, nb_list=(1, 2, 4), k_max=5):
        self.inst = inst
        self.seed = int(seed)
        self.chain = int(chain)
        self.nb = np.ascontiguousarray(nb_list, np.int32)
        self.k_max = int(k_max)
        self.zM = np.ones((inst.K, inst.T), np.uint8)
        self.zR = np.zeros((inst.K, inst.T), np.uint8)
        self.k = 1
        self.it = 0
        self.F, _ = objective(inst, self.zM, self.zR)
        self.F_best = self.F
        self.evals = 0

    def run(self, iters):
        rec = np.zeros(max(int(iters), 1), RECORD_DTYPE)
        k = ctypes.c_int32(self.k)
        fb = ctypes.c_int64(self.F_best)
        ev = ctypes.c_int64(0)
        inst = self.inst
        self.F = int(lib().orc_gvns(inst.K, inst.T, *_inst(inst), self.zM, self.zR, self.nb, len(self.nb),
                                    self.k_max, self.seed, self.chain, self.it, int(iters), ctypes.byref(k),
                                    ctypes.byref(fb), rec, ctypes.byref(ev)))
        self.k = int(k.value)
        self.F_best = int(fb.value)
        self.it += int(iters)
        self.evals += int(ev.value)
        return rec[:int(iters)]


class BestOfChain(Chain):
    """Best-of-G GVNS (Algorithm 2: G shakes of x with the same k, each followed by the VND, the minimum
    selected).  literal=False keeps the GVNS rule of Section 1 (move iff strictly better, k schedule);
    literal=True is Algorithm 2 as printed (k fixed, the minimum always replaces x)."""

    def __init__(self, inst, seed, chain, nb_list=(1, 2, 4), k_max=5, G=2, literal=False):
        super().__init__(inst, seed, chain, nb_list, k_max)
        self.G = int(G)
        self.literal = bool(literal)

    def run(self, iters):
        rec = np.zeros(max(int(iters), 1), RECORD_DTYPE)
        k = ctypes.c_int32(self.k)
        fb = ctypes.c_int64(self.F_best)
        ev = ctypes.c_int64(0)
        inst = self.inst
        self.F = int(lib().orc_gvns_best_of(inst.K, inst.T, *_inst(inst), self.zM, self.zR, self.nb, len(self.nb),
                                            self.k_max, self.G, int(self.literal), self.seed, self.chain, self.it,
                                            int(iters), ctypes.byref(k), ctypes.byref(fb), rec, ctypes.byref(ev)))
        self.k = int(k.value)
        self.F_best = int(fb.value)
        self.it += int(iters)
        self.evals += int(ev.value)
        return rec[:int(iters)]
