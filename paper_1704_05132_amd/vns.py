"""Python binding of libvns.so (the C ABI of include/vns.h): argument marshalling only.

Every step of the search runs in the HIP kernels of the library.  torch is imported first so that the
process holds exactly one HIP runtime (torch's), which the library then shares; torch streams can be bound
to a context with `Context.bind_stream`.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime this library links against)

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libvns.so"

VNS_OK, VNS_EINVAL, VNS_ENOMEM, VNS_EDEVICE, VNS_ERANGE, VNS_ESTATE = 0, -1, -2, -3, -4, -5
NB_FLIP_M, NB_FLIP_R, NB_SHIFT = 1, 2, 4
OPT_CHAINS, OPT_KMAX, OPT_NB_LIST, OPT_TRACE, OPT_RUN_WAVES, OPT_EVAL_GROUP, OPT_RUN_LDS, OPT_GRAPH = 1, 2, 3, 4, 5, 6, 7, 8
OPT_LEARNED, OPT_LOG, OPT_SPECULATE, OPT_SPEC_WAVES, OPT_STATE_LDS, OPT_VND_MEMO = 9, 10, 11, 12, 13, 14
OPT_SPEC_ITERS, OPT_BEST_OF, OPT_BEST_OF_LITERAL, OPT_EVAL_INCREMENTAL, OPT_DECODE = 15, 16, 17, 18, 19
OPT_LEARNED_PACK = 20
OPT_EVAL_SPREAD = 21
DECODE_STRICT, DECODE_DISPOSE = 1, 2
MLP_PARAMS, MLP_FEATURES = 5313, 16
ALL_CHAINS = -1
SOLUTION_CURRENT, SOLUTION_BEST = 0, 1
WS_RUN, WS_EVAL, WS_EVAL_PRICES = 1, 2, 4
INJECT_ALLOC, INJECT_DEVICE = 1, 2
PRICE_INF = np.iinfo(np.int64).max
T_MAX = 128

RECORD_DTYPE = np.dtype([("iter", np.int32), ("k", np.int32), ("accepted", np.int32), ("winner", np.int32),
                         ("F_shaken", np.int64), ("F_local", np.int64), ("F_best", np.int64)])

# Every function the header declares, with its ctypes signature.
_c = ctypes
_P = _c.c_void_p
SIGNATURES = {
    "vns_create": (_c.c_int, [_c.c_int32, _c.c_int32, _P, _P, _P, _P, _P, _P, _c.c_uint64, _c.POINTER(_P)]),
    "vns_create_batch": (_c.c_int, [_c.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _c.c_uint64, _c.POINTER(_P)]),
    "vns_destroy": (None, [_P]),
    "vns_set_option": (_c.c_int, [_P, _c.c_int32, _c.c_int64]),
    "vns_set_unit_costs": (_c.c_int, [_P, _P, _P]),
    "vns_get_option": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int64)]),
    "vns_bind_stream": (_c.c_int, [_P, _P]),
    "vns_workspace_bytes": (_c.c_int, [_P, _c.c_uint32, _c.POINTER(_c.c_size_t)]),
    "vns_bind_workspace": (_c.c_int, [_P, _P, _c.c_size_t, _c.c_uint32]),
    "vns_eval_neighbourhood": (_c.c_int, [_P, _c.c_uint32, _c.c_int32, _P, _P, _P, _P, _P]),
    "vns_eval_neighbourhood_noalloc": (_c.c_int, [_P, _c.c_uint32, _c.c_int32, _P, _P, _P, _P, _P]),
    "vns_run": (_c.c_int, [_P, _c.c_int32]),
    "vns_get_cost": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64)]),
    "vns_get_costs": (_c.c_int, [_P, _P, _P]),
    "vns_get_solution": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _P, _P]),
    "vns_set_solution": (_c.c_int, [_P, _c.c_int32, _P, _P]),
    "vns_get_trajectory": (_c.c_int, [_P, _c.c_int32, _P, _c.c_int64, _c.POINTER(_c.c_int64)]),
    "vns_get_stats": (_c.c_int, [_P, _P]),
    "vns_instance_size": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "vns_mlp_set_params": (_c.c_int, [_P, _P]),
    "vns_mlp_init": (_c.c_int, [_P, _c.c_uint64]),
    "vns_mlp_get_params": (_c.c_int, [_P, _P]),
    "vns_mlp_score": (_c.c_int, [_P, _P, _c.c_int64, _P]),
    "vns_mlp_grad": (_c.c_int, [_P, _P, _P, _c.c_int64, _P, _c.POINTER(_c.c_float)]),
    "vns_mlp_train": (_c.c_int, [_P, _P, _P, _c.c_int64, _c.c_int32, _c.c_int32, _c.c_float, _c.c_uint64,
                                 _c.POINTER(_c.c_float)]),
    "vns_get_move_log": (_c.c_int, [_P, _P, _P, _c.c_int64, _c.POINTER(_c.c_int64)]),
    "vns_eval_learned": (_c.c_int, [_P, _c.c_uint32, _c.c_int32, _c.c_int32, _P, _P, _P, _P, _P]),
    "vns_num_chains": (_c.c_int64, [_P]),
    "vns_last_error": (_c.c_char_p, [_P]),
    "vns_test_inject_failure": (_c.c_int, [_c.c_int32, _c.c_int32]),
}


class VNSStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("move_evals", ctypes.c_int64), ("last_run_evals", ctypes.c_int64),
                ("last_run_ms", ctypes.c_double), ("last_eval_evals", ctypes.c_int64),
                ("last_eval_ms", ctypes.c_double), ("last_run_period_steps", ctypes.c_int64),
                ("last_eval_period_steps", ctypes.c_int64), ("last_run_learned_evals", ctypes.c_int64),
                ("last_run_fallbacks", ctypes.c_int64), ("last_mlp_ms", ctypes.c_double),
                ("last_mlp_rows", ctypes.c_int64), ("last_run_spec_iters", ctypes.c_int64),
                ("last_run_discarded_evals", ctypes.c_int64), ("last_eval_decoded_steps", ctypes.c_int64)]


class VNSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vns status {status}: {msg}")
        self.status = status


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libvns.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1704_05132_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def inject_failure(kind: int, countdown: int):
    """vns_test_inject_failure: make the countdown-th device allocation (INJECT_ALLOC) or call on a live
    context (INJECT_DEVICE) from now fail, on this thread; 0 clears."""
    st = lib().vns_test_inject_failure(int(kind), int(countdown))
    if st != VNS_OK:
        raise VNSError(st, lib().vns_last_error(None).decode())


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Context:
    """A search context: one or several instances, their chains, all state resident on the GPU."""

    def __init__(self, instances, seed: int, chains: int = 1, k_max: int = 5, nb_list: Sequence[int] = (1, 2, 4),
                 trace: bool = True, run_waves: int | None = None, options: dict | None = None):
        L = lib()
        insts = instances if isinstance(instances, (list, tuple)) else [instances]
        self.instances = list(insts)
        h = ctypes.c_void_p()
        if len(insts) == 1:
            D, R, kM, kR, hM, hR = insts[0].arrays()
            self._keep = (D, R, kM, kR, hM, hR)
            st = L.vns_create(insts[0].K, insts[0].T, _ptr(D), _ptr(R), _ptr(kM), _ptr(kR), _ptr(hM), _ptr(hR),
                              ctypes.c_uint64(seed), ctypes.byref(h))
        else:
            K = _i32([i.K for i in insts])
            T = _i32([i.T for i in insts])
            cat = [np.concatenate([np.ravel(i.arrays()[j]) for i in insts]).astype(np.int32) for j in range(6)]
            self._keep = (K, T, *cat)
            st = L.vns_create_batch(len(insts), _ptr(K), _ptr(T), *[_ptr(a) for a in cat], ctypes.c_uint64(seed),
                                    ctypes.byref(h))
        if st != VNS_OK:
            raise VNSError(st, L.vns_last_error(None).decode())
        self.h = h
        self.seed = int(seed)
        if chains != 1:
            self.set_option(OPT_CHAINS, chains)
        if k_max != 5:
            self.set_option(OPT_KMAX, k_max)
        nbv = 0
        for i, nb in enumerate(nb_list):
            nbv |= int(nb) << (4 * i)
        if nbv != 0x421:
            self.set_option(OPT_NB_LIST, nbv)
        if not trace:
            self.set_option(OPT_TRACE, 0)
        if run_waves is not None:
            self.set_option(OPT_RUN_WAVES, run_waves)
        for key, val in (options or {}).items():
            self.set_option(key, val)
        self.chains_per_inst = int(chains)
        models = {(1 if getattr(i, "strict", False) else 0) | (2 if getattr(i, "dispose", False) else 0) for i in insts}
        if len(models) > 1:
            raise ValueError("every instance of a context must take the same decode reading")
        if models != {0}:
            self.set_option(OPT_DECODE, models.pop())
        if any(i.has_unit_costs() for i in insts):
            u = [i.unit_costs() for i in insts]
            self.set_unit_costs(np.concatenate([a for a, _ in u]), np.concatenate([b for _, b in u]))

    # -- plumbing ------------------------------------------------------------------------------------
    def _check(self, st):
        if st != VNS_OK:
            raise VNSError(st, lib().vns_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().vns_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_unit_costs(self, pM, pR):
        """Unit costs of a manufactured / remanufactured item per product (all instances, in order)."""
        a = np.ascontiguousarray(pM, np.int32)
        b = np.ascontiguousarray(pR, np.int32)
        self._check(lib().vns_set_unit_costs(self.h, _ptr(a), _ptr(b)))

    def set_option(self, key, value):
        self._check(lib().vns_set_option(self.h, int(key), int(value)))
        if key == OPT_CHAINS:
            self.chains_per_inst = int(value)

    def get_option(self, key):
        v = ctypes.c_int64()
        self._check(lib().vns_get_option(self.h, int(key), ctypes.byref(v)))
        return int(v.value)

    def bind_stream(self, stream=None):
        """Run on a torch.cuda.Stream (or a raw hipStream_t int); None = the context's own stream."""
        raw = None if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(lib().vns_bind_stream(self.h, ctypes.c_void_p(raw)))

    def workspace_bytes(self, flags: int) -> int:
        n = ctypes.c_size_t()
        self._check(lib().vns_workspace_bytes(self.h, int(flags), ctypes.byref(n)))
        return int(n.value)

    def bind_workspace(self, buf, flags: int):
        """Bind caller-owned device memory (a torch tensor on the context's device, or None to unbind) as the
        workspace of the calls in `flags`; the tensor must stay alive while bound."""
        if buf is None:
            self._check(lib().vns_bind_workspace(self.h, None, 0, 0))
            self._ws = None
            return
        nbytes = buf.numel() * buf.element_size()
        self._check(lib().vns_bind_workspace(self.h, ctypes.c_void_p(buf.data_ptr()), nbytes, int(flags)))
        self._ws = buf

    @property
    def n_chains(self) -> int:
        return int(lib().vns_num_chains(self.h))

    def chain_instance(self, chain: int):
        return self.instances[chain // self.chains_per_inst]

    # -- API -----------------------------------------------------------------------------------------
    def eval_neighbourhood(self, nb_mask: int = 7, chain: int = ALL_CHAINS, slot_prices: bool = True,
                           prod_best: bool = True):
        """Exact prices of every move; returns dict(slot_price, prod_best, prod_best_slot, best, best_slot).
        slot_prices / prod_best = False pass NULL for those outputs (their entries are then None)."""
        chains = range(self.n_chains) if chain == ALL_CHAINS else [chain]
        n_slots = sum(4 * self.chain_instance(g).K * self.chain_instance(g).T for g in chains) if slot_prices else 0
        n_prod = sum(self.chain_instance(g).K for g in chains) if prod_best else 0
        sp = np.empty(n_slots, np.int64) if slot_prices else None
        pb = np.empty(n_prod, np.int64) if prod_best else None
        ps = np.empty(n_prod, np.int32) if prod_best else None
        b = np.empty(len(chains), np.int64)
        bs = np.empty(len(chains), np.int32)
        opt = lambda a: _ptr(a) if a is not None else None
        self._check(lib().vns_eval_neighbourhood(self.h, int(nb_mask), int(chain), opt(sp), opt(pb), opt(ps), _ptr(b),
                                                 _ptr(bs)))
        return dict(slot_price=sp, prod_best=pb, prod_best_slot=ps, best=b, best_slot=bs)

    def eval_neighbourhood_noalloc(self, nb_mask: int = 7, chain: int = ALL_CHAINS, slot_prices: bool = True,
                                   prod_best: bool = True):
        """vns_eval_neighbourhood_noalloc: the same pricing with its scratch in the library's static per-GPU
        array (no allocation); same outputs as eval_neighbourhood."""
        chains = range(self.n_chains) if chain == ALL_CHAINS else [chain]
        n_slots = sum(4 * self.chain_instance(g).K * self.chain_instance(g).T for g in chains) if slot_prices else 0
        n_prod = sum(self.chain_instance(g).K for g in chains) if prod_best else 0
        sp = np.empty(n_slots, np.int64) if slot_prices else None
        pb = np.empty(n_prod, np.int64) if prod_best else None
        ps = np.empty(n_prod, np.int32) if prod_best else None
        b = np.empty(len(chains), np.int64)
        bs = np.empty(len(chains), np.int32)
        opt = lambda a: _ptr(a) if a is not None else None
        self._check(lib().vns_eval_neighbourhood_noalloc(self.h, int(nb_mask), int(chain), opt(sp), opt(pb),
                                                         opt(ps), _ptr(b), _ptr(bs)))
        return dict(slot_price=sp, prod_best=pb, prod_best_slot=ps, best=b, best_slot=bs)

    def run(self, iters: int):
        self._check(lib().vns_run(self.h, int(iters)))

    def cost(self, chain: int):
        F, Fb = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().vns_get_cost(self.h, int(chain), ctypes.byref(F), ctypes.byref(Fb)))
        return int(F.value), int(Fb.value)

    def costs(self):
        """(F, F_best) of every chain as int64 arrays (one copy)."""
        F = np.empty(self.n_chains, np.int64)
        Fb = np.empty(self.n_chains, np.int64)
        self._check(lib().vns_get_costs(self.h, _ptr(F), _ptr(Fb)))
        return F, Fb

    def solution(self, chain: int, which: int = SOLUTION_CURRENT):
        """(zM, zR) [K, T] uint8 of the current solution, or of the best one so far (which = SOLUTION_BEST)."""
        inst = self.chain_instance(chain)
        zM = np.empty((inst.K, inst.T), np.uint8)
        zR = np.empty((inst.K, inst.T), np.uint8)
        self._check(lib().vns_get_solution(self.h, int(chain), int(which), _ptr(zM), _ptr(zR)))
        return zM, zR

    def set_solution(self, chain: int, zM, zR):
        a = np.ascontiguousarray(zM, np.uint8)
        b = np.ascontiguousarray(zR, np.uint8)
        self._check(lib().vns_set_solution(self.h, int(chain), _ptr(a), _ptr(b)))

    def trajectory(self, chain: int):
        n = ctypes.c_int64()
        self._check(lib().vns_get_trajectory(self.h, int(chain), None, 0, ctypes.byref(n)))
        rec = np.zeros(int(n.value), RECORD_DTYPE)
        if len(rec):
            self._check(lib().vns_get_trajectory(self.h, int(chain), _ptr(rec), len(rec), ctypes.byref(n)))
        return rec

    # -- learned scorer ------------------------------------------------------------------------------
    def mlp_set(self, params):
        """params: flat float32[5313] or the list [W1, b1, W2, b2, W3, b3]."""
        flat = np.ascontiguousarray(np.concatenate([np.ravel(p) for p in params]) if isinstance(params, (list, tuple))
                                    else np.ravel(params), np.float32)
        assert flat.size == MLP_PARAMS
        self._check(lib().vns_mlp_set_params(self.h, _ptr(flat)))

    def mlp_init(self, seed: int):
        """He-uniform weights, zero biases, Adam state reset (vns_mlp_init)."""
        self._check(lib().vns_mlp_init(self.h, ctypes.c_uint64(seed)))

    def mlp_get(self):
        out = np.empty(MLP_PARAMS, np.float32)
        self._check(lib().vns_mlp_get_params(self.h, _ptr(out)))
        return out

    def mlp_score(self, feats):
        X = np.ascontiguousarray(feats, np.float32).reshape(-1, MLP_FEATURES)
        out = np.empty(len(X), np.float32)
        self._check(lib().vns_mlp_score(self.h, _ptr(X), len(X), _ptr(out)))
        return out

    def mlp_grad(self, feats, targets):
        X = np.ascontiguousarray(feats, np.float32).reshape(-1, MLP_FEATURES)
        y = np.ascontiguousarray(targets, np.float32)
        g = np.empty(MLP_PARAMS, np.float32)
        loss = ctypes.c_float()
        self._check(lib().vns_mlp_grad(self.h, _ptr(X), _ptr(y), len(X), _ptr(g), ctypes.byref(loss)))
        return float(loss.value), g

    def mlp_train(self, feats, targets, epochs, batch=4096, lr=1e-3, seed=0):
        X = np.ascontiguousarray(feats, np.float32).reshape(-1, MLP_FEATURES)
        y = np.ascontiguousarray(targets, np.float32)
        loss = ctypes.c_float()
        self._check(lib().vns_mlp_train(self.h, _ptr(X), _ptr(y), len(X), int(epochs), int(batch), float(lr),
                                        ctypes.c_uint64(seed), ctypes.byref(loss)))
        return float(loss.value)

    def move_log(self):
        n = ctypes.c_int64()
        self._check(lib().vns_get_move_log(self.h, None, None, 0, ctypes.byref(n)))
        X = np.empty((int(n.value), MLP_FEATURES), np.float32)
        y = np.empty(int(n.value), np.float32)
        if len(y):
            self._check(lib().vns_get_move_log(self.h, _ptr(X), _ptr(y), len(y), ctypes.byref(n)))
        return X, y

    def eval_learned(self, nb, chain, top_permille):
        inst = self.chain_instance(chain)
        n = 4 * inst.K * inst.T
        sc = np.empty(n, np.float32)
        sel = np.empty(n, np.uint8)
        pb = np.empty(inst.K, np.int64)
        ps = np.empty(inst.K, np.int32)
        fb = np.empty(inst.K, np.uint8)
        self._check(lib().vns_eval_learned(self.h, int(nb), int(chain), int(top_permille), _ptr(sc), _ptr(sel),
                                           _ptr(pb), _ptr(ps), _ptr(fb)))
        return dict(scores=sc, selected=sel, prod_best=pb, prod_best_slot=ps, fallback=fb)

    def stats(self) -> dict:
        s = VNSStats()
        self._check(lib().vns_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in VNSStats._fields_}
