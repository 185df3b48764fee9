"""Seeded synthetic instances of the multi-item lot-sizing problem with returns.

The parameters are the ones the paper lists for the problem (Section 2): K products, T periods, demand
D(k,t), returns R(k,t), setup costs kM(k), kR(k) and holding costs hM(k), hR(k). The paper's own
benchmark set (108 instances of 300 products x 52 periods, Section 4) is not available, so every workload
here is synthetic with the distributions below; the int32 arrays this module returns are the contract that
both the CPU oracle and the HIP path consume.

This module draws numbers only: it holds none of the decode, pricing or search arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Instance", "draw_instance", "workload", "WORKLOADS", "edge_instance", "random_pattern"]


@dataclass
class Instance:
    K: int
    T: int
    D: np.ndarray   # int32 [K, T]
    R: np.ndarray   # int32 [K, T]
    kM: np.ndarray  # int32 [K]
    kR: np.ndarray  # int32 [K]
    hM: np.ndarray  # int32 [K]
    hR: np.ndarray  # int32 [K]
    tag: str = field(default="")
    pM: np.ndarray = None   # int32 [K] unit cost of a manufactured item (None: 0)
    pR: np.ndarray = None   # int32 [K] unit cost of a remanufactured item (None: 0)
    strict: bool = False    # decode reading: a remanufacture-only shortfall is infeasible (not carried back)
    dispose: bool = False   # decode reading: returns no lot needs are disposed of (no holding charged on them)

    def arrays(self):
        """(D, R, kM, kR, hM, hR) as C-contiguous int32 arrays."""
        return tuple(np.ascontiguousarray(a, dtype=np.int32)
                     for a in (self.D, self.R, self.kM, self.kR, self.hM, self.hR))

    def unit_costs(self):
        """(pM, pR) as C-contiguous int32 arrays (zeros when not set)."""
        z = np.zeros(self.K, np.int32)
        return (np.ascontiguousarray(self.pM if self.pM is not None else z, dtype=np.int32),
                np.ascontiguousarray(self.pR if self.pR is not None else z, dtype=np.int32))

    def has_unit_costs(self):
        return any(a is not None and np.any(np.asarray(a) != 0) for a in (self.pM, self.pR))

    def product(self, k: int) -> "Instance":
        """The single-product instance made of product k."""
        sl = slice(k, k + 1)
        pM, pR = self.unit_costs()
        return Instance(1, self.T, self.D[sl].copy(), self.R[sl].copy(), self.kM[sl].copy(),
                        self.kR[sl].copy(), self.hM[sl].copy(), self.hR[sl].copy(), f"{self.tag}/p{k}",
                        pM[sl].copy(), pR[sl].copy(), self.strict, self.dispose)


def draw_instance(rng: np.random.Generator, K: int, T: int, ret_lo: float = 0.2, ret_hi: float = 0.8,
                  d_hi: int = 200, tag: str = "") -> Instance:
    """Draw one instance in a fixed order: D, the return fraction u, kM, kR, hM, hR.

    D ~ U{0..d_hi}; R = floor(D * u) with u ~ U(ret_lo, ret_hi) per (k, t), computed once in float64;
    kM, kR ~ U{200..2000}; hM ~ U{2..6}; hR ~ U{1..hM}.
    """
    D = rng.integers(0, d_hi + 1, size=(K, T))
    u = rng.uniform(ret_lo, ret_hi, size=(K, T))
    R = np.floor(D.astype(np.float64) * u).astype(np.int64)
    kM = rng.integers(200, 2001, size=K)
    kR = rng.integers(200, 2001, size=K)
    hM = rng.integers(2, 7, size=K)
    hR = rng.integers(1, hM + 1)
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return Instance(K, T, i32(D), i32(R), i32(kM), i32(kR), i32(hM), i32(hR), tag)


# The five workloads: sizes, neighbourhood lists and seeds.  "nb" lists neighbourhood ids in VND order
# (1 = flip zM, 2 = flip zR, 4 = shift a setup by one period).
WORKLOADS = {
    "plain_10x12": dict(n_inst=1, K=10, T=12, chains=1, iters=500, nb=(1, 2), seed=1,
                        desc="Plain VNS, 1 instance, K=10, T=12, flips only, 1 chain x 500 iterations"),
    "plain_100x52": dict(n_inst=1, K=100, T=52, chains=64, iters=2000, nb=(1, 2, 4), seed=2,
                         desc="Plain VNS, 1 instance, K=100, T=52, 64 Philox chains x 2000 iterations"),
    "batched_4096": dict(n_inst=4096, K=(10, 200), T=(12, 24, 52), chains=8, iters=1000, nb=(1, 2, 4), seed=3,
                         desc="Batched plain VNS, 4096 instances, K~U{10..200}, T in {12,24,52}, 8 chains x 1000"),
    "learned_100x52": dict(n_inst=17, K=100, T=52, chains=64, iters=2000, nb=(1, 2, 4), seed=4,
                           desc="Learned proposal on K=100, T=52 instances"),
    "paper_300x52": dict(n_inst=108, K=300, T=52, chains=8, iters=2000, nb=(1, 2, 4), seed=6,
                         desc="The paper's benchmark shape (108 instances of 300 products x 52 periods), synthetic"),
    "learned_batched_1024": dict(n_inst=1024, K=(100, 1000), T=(52, 104), chains=16, iters=5000,
                                 nb=(1, 2, 4), seed=5, ret=(0.1, 0.9),
                                 desc="Learned + batched, 1024 instances, K~U{100..1000}, T in {52,104}"),
}


def _seq_instance(entropy, K, T, ret=(0.2, 0.8), tag=""):
    rng = np.random.default_rng(np.random.SeedSequence(entropy))
    if isinstance(K, tuple):
        K = int(rng.integers(K[0], K[1] + 1))
    if isinstance(T, tuple):
        T = int(rng.choice(np.array(T)))
    return draw_instance(rng, K, T, ret[0], ret[1], tag=tag)


def workload(name: str, i: int = 0) -> Instance:
    """Instance i of a named workload.

    plain_10x12: SeedSequence(1); plain_100x52: SeedSequence(2); batched_4096: SeedSequence([3, i]) with K then
    T drawn first; learned_100x52: i = 0 is the plain_100x52 instance, i >= 1 SeedSequence([4, i - 1]),
    training instances are i >= 100; learned_batched_1024: SeedSequence([5, i]); paper_300x52: SeedSequence([6, i]),
    instances 0..107 are the set, training instances are i >= 1000.
    """
    w = WORKLOADS[name]
    if name == "plain_10x12":
        return _seq_instance(1, 10, 12, tag=name)
    if name == "plain_100x52":
        return _seq_instance(2, 100, 52, tag=name)
    if name == "batched_4096":
        return _seq_instance([3, i], w["K"], w["T"], tag=f"{name}/{i}")
    if name == "learned_100x52":
        return workload("plain_100x52") if i == 0 else _seq_instance([4, i - 1], 100, 52, tag=f"{name}/{i}")
    if name == "paper_300x52":
        return _seq_instance([6, i], 300, 52, tag=f"{name}/{i}")
    if name == "learned_batched_1024":
        return _seq_instance([5, i], w["K"], w["T"], ret=w["ret"], tag=f"{name}/{i}")
    raise KeyError(name)


def edge_instance(kind: str, K: int, T: int, seed: int = 0) -> Instance:
    """Degenerate instances for edge-case tests.

    kinds: "zero_demand" (D = 0), "no_returns" (R = 0), "returns_eq_demand" (R = D), "big_returns"
    (R up to 3x the demand), "sparse" (most demands zero), "zero_costs" (all setup and holding costs 0),
    "uniform" (the standard distribution).
    """
    rng = np.random.default_rng(np.random.SeedSequence([99, seed, K, T]))
    inst = draw_instance(rng, K, T, tag=f"{kind}/{K}x{T}/{seed}")
    if kind == "zero_demand":
        inst.D[:] = 0
        inst.R[:] = 0
    elif kind == "no_returns":
        inst.R[:] = 0
    elif kind == "returns_eq_demand":
        inst.R[:] = inst.D
    elif kind == "big_returns":
        inst.R[:] = rng.integers(0, 601, size=(K, T)).astype(np.int32)
    elif kind == "sparse":
        mask = rng.random((K, T)) < 0.7
        inst.D[mask] = 0
        inst.R[mask] = 0
    elif kind == "zero_costs":
        inst.kM[:] = 0
        inst.kR[:] = 0
        inst.hM[:] = 0
        inst.hR[:] = 0
    elif kind != "uniform":
        raise KeyError(kind)
    return inst


def random_pattern(inst: Instance, rng: np.random.Generator, p_m: float = 0.3, p_r: float = 0.2):
    """Random setup rows (zM, zR) as [K, T] uint8: zM(k, t) ~ Bernoulli(p_m) with zM(k, 0) = 1 for every product,
    zR(k, t) ~ Bernoulli(p_r), drawn in that order.  A manufacturing setup in the first period makes every
    pattern feasible under the carry-back reading of a remanufacture-only shortfall."""
    zM = (rng.random((inst.K, inst.T)) < p_m).astype(np.uint8)
    zM[:, 0] = 1
    zR = (rng.random((inst.K, inst.T)) < p_r).astype(np.uint8)
    return zM, zR
