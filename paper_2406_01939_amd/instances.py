"""Seeded synthetic fulfillment instances (inputs only; none of the method's arithmetic).

The fulfillment-optimization model of Section 3 has I products (here K SKUs) stocked at
J nodes (here N warehouses); every order carries a product and a reward vector.  The
paper's own data (population-weighted nodes, zip-code distances; Appendix A.3, data
generation) is not available, so every instance here is synthetic:

* SKU of each order: Zipf with exponent 1.1 over K, P(k) proportional to (k+1)^-1.1
  (the heavy-tailed demand shape Q_i ~ i^beta of Section 4.1, with beta = -1.1; the
  `zipf` override sets another exponent, 0 for uniform demand);
* region of each order: uniform over R; the reward of warehouse w for region r is
  -cost[w, r], with integer cost uniform in 1..100 (stands in for the distance reward);
* quantity: 1, or a geometric(p=0.6) law truncated to 1..qmax and renormalised;
* initial inventory x0[k, w] ~ Poisson(0.8 * T * P(k) * E[q] / N): the network holds
  80% of expected demand (Appendix A.3), split evenly over warehouses.  For the largest
  workload (16 x 1e6 SKUs x 500 warehouses = 8e9 values) the draws come from a
  counter-based generator instead, so they can be made on the GPU and any row recomputed
  on the CPU: a 32-bit hash of (seed, trajectory, SKU, warehouse) inverted through the
  Poisson CDF of the SKU (`PoissonX0`);
* learned-policy parameters: PyTorch-default-style uniform init, embedding ~ N(0, 1);
* node capacity (unit-demand workloads): the network can process a fraction of expected
  demand, split evenly: c_1[w] = floor(frac * T / N) (`capacity`).  Appendix A.3 uses 80%;
  at 1e6 orders over 1e5 SKUs the stock already holds shipments to 76% of demand, so no
  node would run out, and that workload uses 60% (every node runs out).

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark; it only draws numbers.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

EMB_DIM = 16
N_FEATURES = 2 + EMB_DIM  # [cost, log1p(inventory), region embedding]

# Named benchmark workloads with their sizes.  T is either an int or a
# (lo, hi) inclusive range drawn per trajectory from `t_seed`.
WORKLOADS: Dict[str, dict] = {
    "greedy_n10_k100_t1e4": dict(N=10, K=100, R=20, T=10_000, qmax=1, n_traj=1,
                                 seed0=1, policy="greedy", block_len=100),
    "greedy_n100_k1e5_t1e6": dict(N=100, K=100_000, R=200, T=1_000_000, qmax=1,
                                  n_traj=1, seed0=2, policy="greedy"),
    "greedy_batch256_n50_k2e4": dict(N=50, K=20_000, R=100, T=(10_000, 1_000_000),
                                     t_seed=3999, qmax=3, n_traj=256, seed0=3000,
                                     policy="greedy"),
    "mlp_batch64_n100_k5e4_t2e5": dict(N=100, K=50_000, R=200, T=200_000, qmax=1,
                                       n_traj=64, seed0=4000, theta_seed=4999,
                                       policy="mlp"),
    # the same two greedy shapes with node capacity (Section 3's full state (x, c))
    "greedy_cap_n10_k100_t1e4": dict(N=10, K=100, R=20, T=10_000, qmax=1, n_traj=1,
                                     seed0=1, policy="greedy", block_len=100, capacity=0.8),
    "greedy_cap_n100_k1e5_t1e6": dict(N=100, K=100_000, R=200, T=1_000_000, qmax=1,
                                      n_traj=1, seed0=2, policy="greedy", capacity=0.6),
    # Section 4.1's instance shape (J = 30 nodes, I = 1e6 products, T = 3e6 orders); the
    # demand exponent is swept with the `zipf` override (beta = -zipf)
    "greedy_n30_k1e6_t3e6": dict(N=30, K=1_000_000, R=200, T=3_000_000, qmax=1, n_traj=1,
                                 seed0=6, policy="greedy"),
    "mlp_batch16_n500_k1e6_t1e7": dict(N=500, K=1_000_000, R=500, T=10_000_000,
                                       qmax=4, n_traj=16, seed0=5000, theta_seed=5999,
                                       policy="mlp", x0_hashed=True),
}

_M32 = 0xFFFFFFFF


def _fmix32(h, xp):
    """MurmurHash3's 32-bit finaliser on non-negative integers below 2^32, for numpy
    (uint64 arrays) and torch (int64 tensors) alike; products wrap mod 2^64 and only their
    low 32 bits are kept."""
    h = h ^ (h >> 16)
    h = (h * 0x85EBCA6B) & _M32
    h = h ^ (h >> 13)
    h = (h * 0xC2B2AE35) & _M32
    return h ^ (h >> 16)


class PoissonX0:
    """Counter-based Poisson draws x0[b, k, w] ~ Poisson(lam_k).

    u = hash(seed, b, k, w) is uniform on 32 bits; x0 = the number of thresholds
    floor(2^32 F_k(j)), j = 0, 1, ..., that are <= u (inverse CDF, F_k the Poisson(lam_k)
    CDF, tables cut where the tail is below 2^-32).  The thresholds of all SKUs are kept in
    one sorted array with SKU k's shifted by k * 2^32, so one search per value finds its
    count."""

    _tables: Dict[bytes, tuple] = {}  # one table per distinct lam vector

    def __init__(self, lam: np.ndarray, seed: int):
        lam = np.asarray(lam, dtype=np.float64)
        self.K = lam.size
        self.seed = int(seed) & _M32
        key = lam.tobytes()
        if key not in PoissonX0._tables:
            from scipy.stats import poisson
            jmax = np.ceil(lam + 12.0 * np.sqrt(lam) + 4.0).astype(np.int64)
            off = np.zeros(self.K + 1, dtype=np.int64)
            off[1:] = np.cumsum(jmax)
            k_of = np.repeat(np.arange(self.K, dtype=np.int64), jmax)
            j = np.arange(int(off[-1]), dtype=np.int64) - off[k_of]
            F = poisson.cdf(j, lam[k_of])
            th = np.minimum(np.floor(F * 4294967296.0), 4294967295.0).astype(np.int64)
            PoissonX0._tables = {key: (off, (k_of << 32) | th)}  # keep the latest only
        self.off, self.table = PoissonX0._tables[key]  # table sorted: SKU-major

    def _u(self, b, k, w, xp):
        hb = _fmix32((self.seed ^ _fmix32(b + 0x9E3779B9, xp)) & _M32, xp)
        h = _fmix32(hb ^ _fmix32(k + 0x7F4A7C15, xp), xp)
        return _fmix32(h ^ _fmix32(w + 0x165667B1, xp), xp)

    def rows(self, b: int, ks: np.ndarray, N: int) -> np.ndarray:
        """x0[b, ks, :] on the CPU (int32 [len(ks), N])."""
        ks = np.asarray(ks, dtype=np.uint64)
        w = np.arange(N, dtype=np.uint64)
        u = self._u(np.uint64(b), ks[:, None], w[None, :], np)
        key = (ks[:, None].astype(np.int64) << 32) | u.astype(np.int64)
        cnt = np.searchsorted(self.table, key, side="right") - self.off[ks.astype(np.int64)][:, None]
        return cnt.astype(np.int32)

    def device(self, b: int, N: int, out, chunk: int = 1 << 17):
        """Fill out (a torch int32 [K, N] tensor on the GPU) with x0[b]."""
        import torch
        dev = out.device
        table = torch.from_numpy(self.table).to(dev)
        off = torch.from_numpy(self.off).to(dev)
        w = torch.arange(N, device=dev, dtype=torch.int64)
        hb = _fmix32((self.seed ^ _fmix32(torch.tensor(b + 0x9E3779B9, dtype=torch.int64, device=dev), torch)) & _M32, torch)
        hw = _fmix32(w + 0x165667B1, torch)
        for k0 in range(0, self.K, chunk):
            k = torch.arange(k0, min(self.K, k0 + chunk), device=dev, dtype=torch.int64)
            h = _fmix32(hb ^ _fmix32(k + 0x7F4A7C15, torch), torch)
            u = _fmix32(h[:, None] ^ hw[None, :], torch)
            key = (k[:, None] << 32) | u
            cnt = torch.searchsorted(table, key, right=True) - off[k][:, None]
            out[k0:k0 + k.numel()] = cnt.to(torch.int32)


@dataclasses.dataclass
class Instance:
    """A batch of independent trajectories, orders concatenated in CSR form."""
    N: int
    K: int
    R: int
    traj_offsets: np.ndarray  # int64 [n_traj + 1]
    sku: np.ndarray           # int32 [sum T]
    region: np.ndarray        # int32 [sum T]
    qty: np.ndarray           # int32 [sum T]
    x0: np.ndarray            # int32 [n_traj, K, N]
    cost: np.ndarray          # int32 [n_traj, N, R]
    rng_seed: int             # Philox key for the learned policy's Gumbel noise
    params: Optional[np.ndarray] = None  # float32 flat learned-policy parameters
    hidden: int = 64
    n_hidden_layers: int = 2
    name: str = ""
    x0_gen: Optional[List["PoissonX0"]] = None  # per trajectory, when x0 is None

    def x0_rows(self, b: int, ks) -> np.ndarray:
        """Initial inventory rows x0[b, ks, :] (from x0 or recomputed by its generator)."""
        if self.x0 is not None:
            return self.x0[b, np.asarray(ks)]
        return self.x0_gen[b].rows(b, np.asarray(ks), self.N)

    @property
    def n_traj(self) -> int:
        return int(self.traj_offsets.shape[0] - 1)

    @property
    def total_orders(self) -> int:
        return int(self.traj_offsets[-1])

    def horizon(self, b: int) -> int:
        return int(self.traj_offsets[b + 1] - self.traj_offsets[b])

    def trajectory(self, b: int) -> "Instance":
        """Trajectory b as a one-trajectory instance (views, no copies)."""
        lo, hi = int(self.traj_offsets[b]), int(self.traj_offsets[b + 1])
        return dataclasses.replace(
            self, traj_offsets=np.array([0, hi - lo], dtype=np.int64),
            sku=self.sku[lo:hi], region=self.region[lo:hi], qty=self.qty[lo:hi],
            x0=None if self.x0 is None else self.x0[b:b + 1], cost=self.cost[b:b + 1],
            x0_gen=None if self.x0_gen is None else [self.x0_gen[b]])


def zipf_probs(K: int, exponent: float = 1.1) -> np.ndarray:
    p = (np.arange(K, dtype=np.float64) + 1.0) ** (-exponent)
    return p / p.sum()


def qty_probs(qmax: int, p: float = 0.6) -> np.ndarray:
    j = np.arange(1, qmax + 1, dtype=np.float64)
    w = p * (1.0 - p) ** (j - 1)
    return w / w.sum()


def param_count(R: int, hidden: int = 64, n_hidden_layers: int = 2) -> int:
    n = R * EMB_DIM + hidden * N_FEATURES + hidden
    if n_hidden_layers == 2:
        n += hidden * hidden + hidden
    return n + hidden + 1


def make_params(R: int, seed: int, hidden: int = 64, n_hidden_layers: int = 2) -> np.ndarray:
    """Flat float32 pack: E[R][16] | W1[H][18] | b1[H] | (W2[H][H] | b2[H]) | w3[H] | b3."""
    rng = np.random.default_rng(seed)
    parts: List[np.ndarray] = [rng.standard_normal((R, EMB_DIM))]
    a1 = 1.0 / np.sqrt(N_FEATURES)
    parts += [rng.uniform(-a1, a1, (hidden, N_FEATURES)), rng.uniform(-a1, a1, hidden)]
    ah = 1.0 / np.sqrt(hidden)
    if n_hidden_layers == 2:
        parts += [rng.uniform(-ah, ah, (hidden, hidden)), rng.uniform(-ah, ah, hidden)]
    parts += [rng.uniform(-ah, ah, hidden), rng.uniform(-ah, ah, 1)]
    out = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert out.size == param_count(R, hidden, n_hidden_layers)
    return out


def make_trajectory(N: int, K: int, R: int, T: int, qmax: int, seed: int,
                    x0_hashed: bool = False, T_orders: Optional[int] = None,
                    zipf: float = 1.1):
    """One trajectory's orders, cost table and initial inventory (the inventory's scale
    follows T; T_orders, if given, is the number of orders drawn; with x0_hashed the
    inventory is returned as its generator; zipf is the demand exponent, 0 = uniform)."""
    rng = np.random.default_rng(seed)
    T_lam = T
    T = T if T_orders is None else int(T_orders)
    pk = zipf_probs(K, zipf)
    cdf = np.cumsum(pk)
    cdf[-1] = 1.0
    sku = np.minimum(np.searchsorted(cdf, rng.random(T), side="right"), K - 1)
    region = rng.integers(0, R, size=T)
    if qmax == 1:
        qty = np.ones(T, dtype=np.int32)
        mean_q = 1.0
    else:
        pq = qty_probs(qmax)
        qcdf = np.cumsum(pq)
        qcdf[-1] = 1.0
        qty = np.minimum(np.searchsorted(qcdf, rng.random(T), side="right"), qmax - 1) + 1
        mean_q = float((np.arange(1, qmax + 1) * pq).sum())
    cost = rng.integers(1, 101, size=(N, R))
    lam = 0.8 * T_lam * pk * mean_q / N
    if x0_hashed:
        x0 = PoissonX0(lam, seed)
    else:
        x0 = rng.poisson(lam[:, None], size=(K, N)).astype(np.int32)
    return (sku.astype(np.int32), region.astype(np.int32), qty.astype(np.int32),
            cost.astype(np.int32), x0)


def make_instance(name: str, **overrides) -> Instance:
    """Build the named workload; keyword overrides shrink it (e.g. T=5000, n_traj=4)."""
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    N, K, R, n_traj, qmax = cfg["N"], cfg["K"], cfg["R"], cfg["n_traj"], cfg["qmax"]
    T = cfg["T"]
    hashed = bool(cfg.get("x0_hashed", False))
    T_orders = cfg.get("T_orders")
    if isinstance(T, tuple):
        lo, hi = T
        Ts = np.random.default_rng(cfg["t_seed"]).integers(lo, hi + 1, size=n_traj)
    else:
        Ts = np.full(n_traj, int(T), dtype=np.int64)
    To = Ts if T_orders is None else np.minimum(Ts, int(T_orders))
    offs = np.zeros(n_traj + 1, dtype=np.int64)
    offs[1:] = np.cumsum(To)
    total = int(offs[-1])
    sku = np.empty(total, np.int32)
    region = np.empty(total, np.int32)
    qty = np.empty(total, np.int32)
    x0 = None if hashed else np.empty((n_traj, K, N), np.int32)
    gens = [] if hashed else None
    cost = np.empty((n_traj, N, R), np.int32)
    for b in range(n_traj):
        s, r, q, c, x = make_trajectory(N, K, R, int(Ts[b]), qmax, cfg["seed0"] + b, hashed,
                                        int(To[b]), float(cfg.get("zipf", 1.1)))
        sl = slice(int(offs[b]), int(offs[b + 1]))
        sku[sl], region[sl], qty[sl] = s, r, q
        cost[b] = c
        if hashed:
            gens.append(x)
        else:
            x0[b] = x
    params = None
    hidden = cfg.get("hidden", 64)
    nhl = cfg.get("n_hidden_layers", 2)
    if cfg["policy"] == "mlp":
        params = make_params(R, cfg["theta_seed"], hidden, nhl)
    rng_seed = (int(cfg.get("theta_seed", 0)) << 32) | int(cfg["seed0"])
    return Instance(N=N, K=K, R=R, traj_offsets=offs, sku=sku, region=region, qty=qty,
                    x0=x0, cost=cost, rng_seed=rng_seed, params=params, hidden=hidden,
                    n_hidden_layers=nhl, name=name, x0_gen=gens)


def capacity(N: int, T: int, frac: float = 0.8) -> np.ndarray:
    """Node capacities c_1 for T unit orders: frac of the demand, split evenly over N."""
    return np.full(N, int(np.floor(frac * T / N)), dtype=np.int32)


def bid_prices(K: int, N: int, seed: int, spread: int = 50):
    """Fixed dual prices for the bid-price policy with capacity: (bid_inv [K][N], the price
    of a unit of each SKU's stock at each node; bid_cap [N], the price of a unit of each
    node's capacity), int32 uniform on 0..spread (costs are 1..100)."""
    rng = np.random.default_rng(60_000 + seed)
    return (rng.integers(0, spread + 1, (K, N)).astype(np.int32),
            rng.integers(0, spread + 1, N).astype(np.int32))


def workload_capacity(name: str) -> np.ndarray:
    """The node capacities of a named capacity workload."""
    cfg = WORKLOADS[name]
    return capacity(cfg["N"], int(cfg["T"]), cfg["capacity"])


def random_tiny(seed: int, N: int = 4, K: int = 3, R: int = 3, T: int = 12, qmax: int = 1,
                inv_max: int = 3, n_traj: int = 1, mlp: bool = False,
                n_hidden_layers: int = 2) -> Instance:
    """Small random instances for brute-force checks (uniform SKUs, small inventories)."""
    rng = np.random.default_rng(seed)
    Ts = rng.integers(max(1, T // 2), T + 1, size=n_traj) if n_traj > 1 else np.array([T])
    offs = np.zeros(n_traj + 1, dtype=np.int64)
    offs[1:] = np.cumsum(Ts)
    total = int(offs[-1])
    sku = rng.integers(0, K, total).astype(np.int32)
    region = rng.integers(0, R, total).astype(np.int32)
    qty = rng.integers(1, qmax + 1, total).astype(np.int32)
    x0 = rng.integers(0, inv_max + 1, (n_traj, K, N)).astype(np.int32)
    cost = rng.integers(1, 6, (n_traj, N, R)).astype(np.int32)
    params = make_params(R, seed + 7919, 64, n_hidden_layers) if mlp else None
    return Instance(N=N, K=K, R=R, traj_offsets=offs, sku=sku, region=region, qty=qty,
                    x0=x0, cost=cost, rng_seed=int(rng.integers(0, 2**63)), params=params,
                    n_hidden_layers=n_hidden_layers, name=f"tiny{seed}")


# ---------------------------------------------------------------- OWMR inventory problem
# One central warehouse and N retailers (the appendix's inventory-control extension): each
# order is a demand at one retailer; retailers follow (s_n, S_n) order-up-to rules within
# their capacity, the central warehouse an (s, S) rule.  The base case follows the
# appendix's experiment: 4,000 stores, one year of 10,000 units a day as unit demands
# (T = 3.65e6), stores ordering up to 20 when they fall to 10, and a central level that
# lasts about a week (70,000 units); stores are drawn with weights (1 - alpha)^i.
OWMR_WORKLOADS: Dict[str, dict] = {
    "owmr_n4000_t3650000": dict(N=4000, T=3_650_000, s_ret=10, S_ret=20, cap=20, s0=10,
                                S0=70_000, alpha=0.0, dmax=1, seed=7),
    "owmr_n40_t10000": dict(N=40, T=10_000, s_ret=3, S_ret=8, cap=8, s0=10, S0=700,
                            alpha=0.0, dmax=1, seed=8),
}


@dataclasses.dataclass
class OwmrInstance:
    N: int
    retailer: np.ndarray  # int32 [T]
    demand: np.ndarray    # int32 [T]
    s_ret: np.ndarray     # int32 [N] reorder point
    S_ret: np.ndarray     # int32 [N] order-up-to level
    cap: np.ndarray       # int32 [N] capacity
    x_init: np.ndarray    # int32 [N] stock at t = 0
    s0: int
    S0: int
    x0_init: int
    name: str = ""

    @property
    def T(self) -> int:
        return int(self.retailer.size)


def make_owmr_instance(name: str, **overrides) -> OwmrInstance:
    """Build the named OWMR workload; overrides change its sizes or parameters."""
    cfg = dict(OWMR_WORKLOADS[name])
    cfg.update(overrides)
    N, T = int(cfg["N"]), int(cfg["T"])
    rng = np.random.default_rng(cfg["seed"])
    w = (1.0 - float(cfg["alpha"])) ** np.arange(N, dtype=np.float64)
    cdf = np.cumsum(w / w.sum())
    cdf[-1] = 1.0
    retailer = np.minimum(np.searchsorted(cdf, rng.random(T), side="right"), N - 1)
    demand = rng.integers(1, int(cfg["dmax"]) + 1, T)
    full = lambda v: np.full(N, int(v), dtype=np.int32)
    return OwmrInstance(N=N, retailer=retailer.astype(np.int32), demand=demand.astype(np.int32),
                        s_ret=full(cfg["s_ret"]), S_ret=full(cfg["S_ret"]), cap=full(cfg["cap"]),
                        x_init=full(min(cfg["S_ret"], cfg["cap"])), s0=int(cfg["s0"]),
                        S0=int(cfg["S0"]), x0_init=int(cfg["S0"]), name=name)


def random_owmr(seed: int, N: int = 4, T: int = 40, dmax: int = 3, cap_max: int = 6,
                s0=None, S0=None) -> OwmrInstance:
    """Small random OWMR instances for brute-force checks: random retailer levels and
    capacities, demands 0..dmax, a central level a few retailer orders deep."""
    rng = np.random.default_rng(seed)
    cap = rng.integers(1, cap_max + 1, N)
    S_ret = rng.integers(0, cap + 3)  # a level above capacity is cut to it by the policy
    s_ret = rng.integers(-1, S_ret + 1)
    x_init = rng.integers(0, cap + 1)
    S0 = int(rng.integers(cap.max(), 4 * cap.sum() + 2)) if S0 is None else int(S0)
    s0 = int(rng.integers(-1, S0 // 2 + 1)) if s0 is None else int(s0)
    i32 = lambda a: np.asarray(a, dtype=np.int32)
    return OwmrInstance(N=N, retailer=i32(rng.integers(0, N, T)), demand=i32(rng.integers(0, dmax + 1, T)),
                        s_ret=i32(s_ret), S_ret=i32(S_ret), cap=i32(cap), x_init=i32(x_init),
                        s0=s0, S0=S0, x0_init=int(rng.integers(0, S0 + 1)), name=f"owmr{seed}")
