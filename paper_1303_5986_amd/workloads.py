"""Reaction networks and seeded synthetic workloads.

This module only *describes* inputs: species, reactions, rate constants, bin
grids, recycling targets and seeds.  It holds none of the simulation
arithmetic, so both the HIP library and the CPU oracle can be fed from it.

Models:
  * birth-death: 0 -> X (k = 1.0), X -> 0 (gamma = 0.025 per copy); stationary
    law Poisson(40).
  * Schloegl (Sec. III.B, Eq. schlogl): A + 2X <-> 3X, B <-> X with
    k1 = 3e-7, k2 = 1e-4, k3 = 1e-3, k4 = 3.5, A = 1e5, B = 2e5 held constant
    and folded into the rate constants.
  * futile cycle (Sec. III.A, Eq. futile): E1 + S1 <-> B1 -> E1 + S2,
    E2 + S2 <-> B2 -> E2 + S1, k_f = 1.0, k_s = 0.1.
  * the epigenetic switch (Sec. III.C): two genes repressing each other,
    births at Hill-type rates a1 / (1 + (g2/K2)^n), a2 / (1 + (g1/K1)^m),
    a1 = 156, a2 = 30, n = 3, m = 1, K1 = K2 = 1, deaths at 1/tau = 1 per
    copy, on the paper's 15 x 31 two-dimensional bin grid;
  * a synthetic two-gene toggle (8 species, 16 mass-action reactions), and
    synthetic large mass-action networks shaped like the 354-species /
    3680-reaction model of Sec. III.D, both generated from a seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Network:
    """A reaction network in CSR form.

    reactants of reaction j: reac_species[reac_ptr[j]:reac_ptr[j+1]] with
    multiplicities reac_mult (1..3); net change of reaction j:
    chg_species/chg_delta over chg_ptr; rate[j] is the stochastic rate
    constant c_j, with constant reservoir species folded in.  Optionally a
    reaction's mass-action propensity is divided by a repressive Hill factor
    1 + (x_r / K)^n: hill_species[j] = r (-1: none), hill_n[j], hill_K[j].
    """

    S: int
    R: int
    reac_ptr: np.ndarray
    reac_species: np.ndarray
    reac_mult: np.ndarray
    chg_ptr: np.ndarray
    chg_species: np.ndarray
    chg_delta: np.ndarray
    rate: np.ndarray
    names: List[str]
    hill_species: Optional[np.ndarray] = None
    hill_n: Optional[np.ndarray] = None
    hill_K: Optional[np.ndarray] = None

    @property
    def has_hill(self) -> bool:
        return self.hill_species is not None and bool((self.hill_species >= 0).any())

    @staticmethod
    def from_reactions(names: Sequence[str], reactions: Sequence[tuple]) -> "Network":
        """Build from (reactants, products, c_j) triples, or quadruples whose
        last entry is a Hill factor (species name, n, K); reactants and
        products map species name -> stoichiometric count."""
        idx = {n: i for i, n in enumerate(names)}
        rp, rs, rm, cp, cs, cd, rate = [0], [], [], [0], [], [], []
        hs, hn, hk = [], [], []
        for rx in reactions:
            reac, prod, c = rx[0], rx[1], rx[2]
            hill = rx[3] if len(rx) > 3 else None
            hs.append(idx[hill[0]] if hill else -1)
            hn.append(int(hill[1]) if hill else 0)
            hk.append(float(hill[2]) if hill else 0.0)
            for sp in sorted(reac, key=lambda n: idx[n]):
                rs.append(idx[sp])
                rm.append(int(reac[sp]))
            rp.append(len(rs))
            delta: Dict[int, int] = {}
            for sp, k in reac.items():
                delta[idx[sp]] = delta.get(idx[sp], 0) - int(k)
            for sp, k in prod.items():
                delta[idx[sp]] = delta.get(idx[sp], 0) + int(k)
            for s in sorted(delta):
                if delta[s] != 0:
                    cs.append(s)
                    cd.append(delta[s])
            cp.append(len(cs))
            rate.append(float(c))
        i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32))
        any_hill = any(v >= 0 for v in hs)
        return Network(S=len(names), R=len(reactions),
                       reac_ptr=i32(rp), reac_species=i32(rs), reac_mult=i32(rm),
                       chg_ptr=i32(cp), chg_species=i32(cs), chg_delta=i32(cd),
                       rate=np.ascontiguousarray(np.asarray(rate, dtype=np.float64)),
                       names=list(names),
                       hill_species=i32(hs) if any_hill else None,
                       hill_n=i32(hn) if any_hill else None,
                       hill_K=np.ascontiguousarray(np.asarray(hk, np.float64)) if any_hill else None)

    def order(self, j: int) -> int:
        return int(self.reac_mult[self.reac_ptr[j]:self.reac_ptr[j + 1]].sum())


@dataclasses.dataclass
class WEConfig:
    """Everything the WE procedure needs besides the network: the bin grid on
    a linear progress coordinate (or on two, bin = b1 + n1 * b2), walkers per
    bin, the interval, the initial state, the recycling target and the seeds
    of independent runs."""

    name: str
    net: Network
    x0: np.ndarray                 # int32[S]
    bin_coef: np.ndarray           # float64[S]
    edges: np.ndarray              # float64[n_bins + 1]
    m_targ: int
    tau: float
    n_iters: int
    seeds: np.ndarray              # uint64[n_runs]
    recycle: bool = False
    tgt_coef: Optional[np.ndarray] = None
    tgt_thr: float = 0.0
    x_rec: Optional[np.ndarray] = None
    hist_species: int = 0
    hist_lo: int = 0
    hist_hi: int = 0
    bin_coef2: Optional[np.ndarray] = None   # second grid axis (None: 1-D)
    edges2: Optional[np.ndarray] = None
    engine: str = "ssa"                      # "ssa" (exact) or "tauleap"
    leap_eps: float = 0.03                   # tau-leaping error control
    resample_rule: int = 0                   # 0: count-only split/merge as printed;
                                             # 1: weight-equalizing (keeps a bin's weights
                                             #    near its weight / m_targ)

    @property
    def n_bins1(self) -> int:
        return len(self.edges) - 1

    @property
    def n_bins2(self) -> int:
        return 1 if self.edges2 is None else len(self.edges2) - 1

    @property
    def n_bins(self) -> int:
        return self.n_bins1 * self.n_bins2

    @property
    def cap(self) -> int:
        return self.m_targ * self.n_bins

    def with_seeds(self, seeds) -> "WEConfig":
        return dataclasses.replace(self, seeds=np.asarray(seeds, dtype=np.uint64))


def uniform_edges(lo: float, hi: float, n: int) -> np.ndarray:
    """n equal bins on [lo, hi]: edges lo + i*(hi-lo)/n."""
    return np.array([lo + i * (hi - lo) / n for i in range(n + 1)], dtype=np.float64)


# --------------------------------------------------------------------------
# 1-D birth-death.
# --------------------------------------------------------------------------
def birth_death(k: float = 1.0, gamma: float = 0.025) -> Network:
    return Network.from_reactions(["X"], [({}, {"X": 1}, k), ({"X": 1}, {}, gamma)])


def birth_death_config(n_runs: int = 1, seed0: int = 1, n_iters: int = 200) -> WEConfig:
    net = birth_death()
    return WEConfig(
        name="birth_death", net=net, x0=np.array([40], np.int32),
        bin_coef=np.array([1.0]), edges=uniform_edges(0.0, 120.0, 20),
        m_targ=4, tau=1.0, n_iters=n_iters,
        seeds=np.arange(seed0, seed0 + n_runs, dtype=np.uint64),
        hist_species=0, hist_lo=0, hist_hi=140)


# --------------------------------------------------------------------------
# Schloegl model, Sec. III.B.
# --------------------------------------------------------------------------
SCHLOGL_K = dict(k1=3e-7, k2=1e-4, k3=1e-3, k4=3.5, A=1e5, B=2e5)


def schlogl() -> Network:
    p = SCHLOGL_K
    return Network.from_reactions(["X"], [
        ({"X": 2}, {"X": 3}, p["k1"] * p["A"]),      # A + 2X -> 3X
        ({"X": 3}, {"X": 2}, p["k2"]),               # 3X -> A + 2X
        ({}, {"X": 1}, p["k3"] * p["B"]),            # B -> X
        ({"X": 1}, {}, p["k4"]),                     # X -> B
    ])


def schlogl_config(n_runs: int = 1, seed0: int = 1, n_iters: int = 2000,
                   recycle: bool = True) -> WEConfig:
    """60 bins of width 40/3 on [0, 800], 8 walkers per bin, tau = 0.05;
    steady state with recycling X >= 563 -> X = 82 (the two wells of
    Sec. III.B)."""
    net = schlogl()
    return WEConfig(
        name="schlogl", net=net, x0=np.array([82], np.int32),
        bin_coef=np.array([1.0]), edges=uniform_edges(0.0, 800.0, 60),
        m_targ=8, tau=0.05, n_iters=n_iters,
        seeds=np.arange(seed0, seed0 + n_runs, dtype=np.uint64),
        recycle=recycle, tgt_coef=np.array([1.0]), tgt_thr=563.0,
        x_rec=np.array([82], np.int32),
        hist_species=0, hist_lo=0, hist_hi=800)


# --------------------------------------------------------------------------
# Enzymatic futile cycle, Sec. III.A.
# --------------------------------------------------------------------------
def futile_cycle(kf: float = 1.0, ks: float = 0.1) -> Network:
    names = ["S1", "S2", "E1", "E2", "B1", "B2"]
    return Network.from_reactions(names, [
        ({"E1": 1, "S1": 1}, {"B1": 1}, kf),
        ({"B1": 1}, {"E1": 1, "S1": 1}, kf),
        ({"B1": 1}, {"E1": 1, "S2": 1}, ks),
        ({"E2": 1, "S2": 1}, {"B2": 1}, kf),
        ({"B2": 1}, {"E2": 1, "S2": 1}, kf),
        ({"B2": 1}, {"E2": 1, "S1": 1}, ks),
    ])


# --------------------------------------------------------------------------
# Small test networks.
# --------------------------------------------------------------------------
def isomerization(k_ab: float = 1.0, k_ba: float = 0.5) -> Network:
    """A <-> B: with N molecules the stationary law of A is Binomial."""
    return Network.from_reactions(["A", "B"], [({"A": 1}, {"B": 1}, k_ab),
                                               ({"B": 1}, {"A": 1}, k_ba)])


# --------------------------------------------------------------------------
# Seeded random mass-action networks shaped like the 354-species /
# 3680-reaction model of Sec. III.D.
# --------------------------------------------------------------------------
def random_network(seed: int, S: int = 354, R: int = 3680, frac_zeroth: float = 0.1,
                   frac_uni: float = 0.4, rate_lo: float = 1e-4, rate_hi: float = 1e1) -> Network:
    """A random mass-action network from a seed.

    * every species decays, X -> 0 (part of the unimolecular share), so every
      species has an outflow;
    * species carry masses m in {1,2,3}; every reaction with reactants keeps
      sum(m products) <= sum(m reactants), so only the zeroth-order inflows
      0 -> X add mass and copy numbers stay bounded;
    * unimolecular X -> Y | Y + Z, bimolecular X + Y -> Z | Z + W (homodimers
      X + X allowed), zeroth order 0 -> X | X + Y, no duplicate reactions;
    * rate constants log-uniform on [rate_lo, rate_hi].
    """
    rng = np.random.default_rng(seed)
    mass = rng.integers(1, 4, size=S)
    names = [f"s{i}" for i in range(S)]
    n0 = int(round(frac_zeroth * R))
    n1 = max(int(round(frac_uni * R)), S)      # at least one decay per species
    n2 = R - n0 - n1
    if n2 < 0:
        raise ValueError("need at least one unimolecular reaction per species (decays)")
    seen = set()
    reactions = []

    def rate():
        return float(np.exp(rng.uniform(np.log(rate_lo), np.log(rate_hi))))

    def add(reac: Dict[str, int], prod: Dict[str, int]) -> bool:
        key = (tuple(sorted(reac.items())), tuple(sorted(prod.items())))
        if key in seen or reac == prod:
            return False
        seen.add(key)
        reactions.append((reac, prod, rate()))
        return True

    def products_within(budget: int) -> Dict[str, int]:
        # zero, one or two product molecules whose total mass fits the budget
        choice = rng.integers(0, 3)
        prod: Dict[str, int] = {}
        if choice == 0:
            return prod
        cand = np.flatnonzero(mass <= budget)
        if len(cand) == 0:
            return prod
        a = int(rng.choice(cand))
        prod[names[a]] = 1
        if choice == 2:
            cand2 = np.flatnonzero(mass <= budget - mass[a])
            if len(cand2):
                b = int(rng.choice(cand2))
                prod[names[b]] = prod.get(names[b], 0) + 1
        return prod

    def give_up(tries):
        if tries > 200000:
            raise ValueError(f"cannot draw {R} distinct reactions over {S} species")
        return tries + 1

    for s in range(S):
        add({names[s]: 1}, {})
    tries = 0
    while len(reactions) < n1:
        tries = give_up(tries)
        s = int(rng.integers(0, S))
        prod = products_within(int(mass[s]))
        if not prod:
            continue
        add({names[s]: 1}, prod)
    while len(reactions) < n1 + n2:
        tries = give_up(tries)
        a, b = (int(v) for v in rng.integers(0, S, size=2))
        reac = {names[a]: 2} if a == b else {names[a]: 1, names[b]: 1}
        add(reac, products_within(int(mass[a] + mass[b])))
    while len(reactions) < R:
        tries = give_up(tries)
        # inflow of one molecule, or of two once single inflows run out
        a, b = (int(v) for v in rng.integers(0, S, size=2))
        prod = {names[a]: 1} if rng.random() < 0.5 or len(reactions) - n1 - n2 >= S // 2 \
            else ({names[a]: 2} if a == b else {names[a]: 1, names[b]: 1})
        add({}, prod)
    net = Network.from_reactions(names, reactions)
    net.mass = mass
    return net


def log_uniform_counts(rng: np.random.Generator, S: int, hi: int = 1000) -> np.ndarray:
    """floor(exp(U[0, ln(hi+1)])) - 1, i.e. counts on [0, hi], log-uniform."""
    return (np.floor(np.exp(rng.uniform(0.0, np.log(hi + 1.0), size=S))) - 1).astype(np.int32)


def producing_counts(net: Network) -> np.ndarray:
    """Number of reactions that increase each species."""
    c = np.zeros(net.S, np.int64)
    for j in range(net.R):
        for p in range(net.chg_ptr[j], net.chg_ptr[j + 1]):
            if net.chg_delta[p] > 0:
                c[net.chg_species[p]] += 1
    return c


def first_order_loss(net: Network) -> np.ndarray:
    """kappa_s: summed rate constants of the unimolecular reactions that
    consume species s (weighted by copies consumed)."""
    k = np.zeros(net.S)
    for j in range(net.R):
        if net.order(j) != 1:
            continue
        for p in range(net.chg_ptr[j], net.chg_ptr[j + 1]):
            if net.chg_delta[p] < 0:
                k[net.chg_species[p]] += net.rate[j] * (-net.chg_delta[p])
    return k


def large_network_config(seed: int = 2024, n_walkers: int = 4096, n_bins: int = 50,
                         n_iters: int = 50, tau: float = 0.1, S: int = 354,
                         R: int = 3680) -> WEConfig:
    """Synthetic stand-in for the 354/3680 model of Sec. III.D: seeded network,
    log-uniform initial counts on [0, 1000], 50 bins of width 20 on [0, 1000),
    floor(4096/50) = 81 walkers per bin, tau = 0.1.

    The binned species is the one with the largest x0_s * exp(-kappa_s * 1 s)
    (kappa_s its first-order loss constant): a structural rule that picks a
    species present in hundreds of copies and slow to decay, so the 50 bins
    are actually visited.  The joint histogram takes the next four by the
    same score."""
    net = random_network(seed, S, R)
    rng = np.random.default_rng(seed + 1)
    x0 = log_uniform_counts(rng, S)
    score = x0 * np.exp(-first_order_loss(net))
    order = sorted(range(S), key=lambda s: (-score[s], s))
    bs = order[0]
    coef = np.zeros(S)
    coef[bs] = 1.0
    cfg = WEConfig(name="large_network", net=net, x0=x0, bin_coef=coef,
                   edges=uniform_edges(0.0, 1000.0, n_bins), m_targ=n_walkers // n_bins, tau=tau,
                   n_iters=n_iters, seeds=np.array([seed], np.uint64),
                   hist_species=bs, hist_lo=0, hist_hi=1000)
    cfg.joint_species = order[:5]
    return cfg


# --------------------------------------------------------------------------
# Synthetic two-gene mutual-repression toggle (8 species, 16 reactions).
# --------------------------------------------------------------------------
TOGGLE_SPECIES = ["G1", "G1r", "G2", "G2r", "P1", "P2", "D1", "D2"]


# --------------------------------------------------------------------------
# Epigenetic switch, Sec. III.C.
# --------------------------------------------------------------------------
SWITCH_P = dict(a1=156.0, a2=30.0, n=3, m=1, K1=1.0, K2=1.0, k0=1.0)


def switch() -> Network:
    """0 -> g1 at a1 / (1 + (g2/K2)^n), g1 -> 0 at k0 g1, 0 -> g2 at
    a2 / (1 + (g1/K1)^m), g2 -> 0 at k0 g2 (Sec. III.C)."""
    p = SWITCH_P
    return Network.from_reactions(["g1", "g2"], [
        ({}, {"g1": 1}, p["a1"], ("g2", p["n"], p["K2"])),
        ({"g1": 1}, {}, p["k0"]),
        ({}, {"g2": 1}, p["a2"], ("g1", p["m"], p["K1"])),
        ({"g2": 1}, {}, p["k0"]),
    ])


def switch_config(n_runs: int = 6, seed0: int = 1, n_iters: int = 500, m_targ: int = 16) -> WEConfig:
    """The WE setup of Sec. III.C: 15 bins on g1 (unit width on [0, 10],
    width 10 on [10, 50], then [50, inf)) times 31 on g2 (unit width on
    [0, 30], then [30, inf)); 16 walkers per bin; tau = 0.1.  States (never
    defined in the paper): A = (g1, g2) = (0, 30), the g2-high state, and
    B = {g1 >= 50}; walkers reaching B restart from A."""
    top = 1e9
    e1 = np.array(list(range(0, 11)) + [20, 30, 40, 50, top], np.float64)
    e2 = np.array(list(range(0, 31)) + [top], np.float64)
    return WEConfig(
        name="switch", net=switch(), x0=np.array([0, 30], np.int32),
        bin_coef=np.array([1.0, 0.0]), edges=e1, m_targ=m_targ, tau=0.1, n_iters=n_iters,
        seeds=np.arange(seed0, seed0 + n_runs, dtype=np.uint64),
        recycle=True, tgt_coef=np.array([1.0, 0.0]), tgt_thr=50.0,
        x_rec=np.array([0, 30], np.int32),
        bin_coef2=np.array([0.0, 1.0]), edges2=e2)


def toggle_rates(seed: int) -> Dict[str, float]:
    """Eight rate constants log-uniform on [1e-3, 10], shared by the two
    mirror-image genes; the leak is the smaller of the two expression draws."""
    rng = np.random.default_rng(seed)
    r = np.exp(rng.uniform(np.log(1e-3), np.log(1e1), 8))
    ke, kl, kp, kd, ku, kb, kub, kdd = (float(v) for v in r)
    if kl > ke:
        ke, kl = kl, ke
    return dict(ke=ke, kl=kl, kp=kp, kd=kd, ku=ku, kb=kb, kub=kub, kdd=kdd)


def toggle(p: Dict[str, float]) -> Network:
    """Expression G -> G + P, leak Gr -> Gr + P, P -> 0, 2P -> D, D -> 2P,
    promoter binding G1 + D2 -> G1r (and mirror), unbinding, D -> 0."""
    R = [({"G1": 1}, {"G1": 1, "P1": 1}, p["ke"]), ({"G2": 1}, {"G2": 1, "P2": 1}, p["ke"]),
         ({"G1r": 1}, {"G1r": 1, "P1": 1}, p["kl"]), ({"G2r": 1}, {"G2r": 1, "P2": 1}, p["kl"]),
         ({"P1": 1}, {}, p["kp"]), ({"P2": 1}, {}, p["kp"]),
         ({"P1": 2}, {"D1": 1}, p["kd"]), ({"P2": 2}, {"D2": 1}, p["kd"]),
         ({"D1": 1}, {"P1": 2}, p["ku"]), ({"D2": 1}, {"P2": 2}, p["ku"]),
         ({"G1": 1, "D2": 1}, {"G1r": 1}, p["kb"]), ({"G2": 1, "D1": 1}, {"G2r": 1}, p["kb"]),
         ({"G1r": 1}, {"G1": 1, "D2": 1}, p["kub"]), ({"G2r": 1}, {"G2": 1, "D1": 1}, p["kub"]),
         ({"D1": 1}, {}, p["kdd"]), ({"D2": 1}, {}, p["kdd"])]
    return Network.from_reactions(TOGGLE_SPECIES, R)


def _toggle_rre_states(p: Dict[str, float]):
    """Steady states of the reaction-rate equations reached from gene-1-on and
    gene-2-on starts (gene occupancies as fractions)."""
    from scipy.integrate import solve_ivp

    def rhs(t, y):
        G1r, G2r, P1, P2, D1, D2 = y
        G1, G2 = 1 - G1r, 1 - G2r
        return [p["kb"] * G1 * D2 - p["kub"] * G1r,
                p["kb"] * G2 * D1 - p["kub"] * G2r,
                p["ke"] * G1 + p["kl"] * G1r - p["kp"] * P1 - p["kd"] * P1 * P1 + 2 * p["ku"] * D1,
                p["ke"] * G2 + p["kl"] * G2r - p["kp"] * P2 - p["kd"] * P2 * P2 + 2 * p["ku"] * D2,
                p["kd"] * P1 * P1 / 2 - (p["ku"] + p["kdd"]) * D1 - p["kb"] * G2 * D1 + p["kub"] * G2r,
                p["kd"] * P2 * P2 / 2 - (p["ku"] + p["kdd"]) * D2 - p["kb"] * G1 * D2 + p["kub"] * G1r]

    out = []
    for y0 in ([0, 1, 50, 0, 50, 0], [1, 0, 0, 50, 0, 50]):
        s = solve_ivp(rhs, (0, 2e4), y0, method="LSODA", rtol=1e-8, atol=1e-10)
        out.append(s.y[:, -1])
    return out   # [gene-1-on state, gene-2-on state]


def toggle_accepts(p: Dict[str, float]) -> bool:
    """Two distinct stable states (mirror images, |Delta| > 20 where
    Delta = (P1 + 2 D1) - (P2 + 2 D2)) with every count at most 500."""
    b, a = _toggle_rre_states(p)
    da = (a[2] + 2 * a[4]) - (a[3] + 2 * a[5])
    db = (b[2] + 2 * b[4]) - (b[3] + 2 * b[5])
    return da < -20 and db > 20 and max(a[2:].max(), b[2:].max()) <= 500


def toggle_config(seed0: int = 100, n_runs: int = 16, n_bins: int = 64, m_targ: int = 16,
                  n_iters: int = 500, tau: float = 0.7) -> WEConfig:
    """The first seed >= seed0 whose rates pass toggle_accepts (seed 101 for
    seed0 = 100).  A = the rounded gene-2-on steady state (walkers restart
    there), B = {Delta >= 0.8 Delta_B*} with Delta_B* the gene-1-on value;
    64 plain bins on Delta over [Delta_A - 8, threshold); tau = 0.7, about
    10 / a0 at A (a0(A) = 14.85 for seed 101: ten reactions per walker and
    interval)."""
    seed = seed0
    while not toggle_accepts(toggle_rates(seed)):
        seed += 1
    p = toggle_rates(seed)
    b, a = _toggle_rre_states(p)
    xA = np.array([round(1 - a[0]), round(a[0]), round(1 - a[1]), round(a[1]),
                   round(a[2]), round(a[3]), round(a[4]), round(a[5])], np.int32)
    dB = (b[2] + 2 * b[4]) - (b[3] + 2 * b[5])
    thr = float(np.floor(0.8 * dB))
    coef = np.array([0, 0, 0, 0, 1, -1, 2, -2], np.float64)
    dA = float(coef @ xA)
    net = toggle(p)
    cfg = WEConfig(name="toggle", net=net, x0=xA, bin_coef=coef,
                   edges=uniform_edges(dA - 8.0, thr, n_bins), m_targ=m_targ, tau=tau,
                   n_iters=n_iters, seeds=np.arange(1, n_runs + 1, dtype=np.uint64),
                   recycle=True, tgt_coef=coef.copy(), tgt_thr=thr, x_rec=xA.copy(),
                   hist_species=4, hist_lo=0, hist_hi=200)
    cfg.toggle_seed = seed
    cfg.a_thr = -thr          # A region for committor labels: Delta <= -thr
    return cfg


# --------------------------------------------------------------------------
# A batch of independent runs on networks of uneven size.
# --------------------------------------------------------------------------
def batch_configs(n_runs: int = 64, seed: int = 7, r_max: int = 3680, w_min: int = 256,
                  w_max: int = 8192, n_bins: int = 16, tau: float = 0.01,
                  n_iters: int = 200) -> List[WEConfig]:
    """Run k of n: R_k = round(8 * (r_max/8)^(k/(n-1))) reactions,
    S_k = max(round(R_k * 354/3680), min(8, R_k // 3)) species (the floor
    leaves the smallest networks enough species to draw distinct reactions
    under the mass rule), walker slots
    W_k = w_min * (w_max/w_min)^(pi(k)/(n-1)) with pi a seeded permutation
    (so network size and walker count are not correlated), 16 bins on the
    species chosen by the same structural rule as the large network, initial
    counts log-uniform on [0, 20], no recycling."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_runs)
    out = []
    for k in range(n_runs):
        f = k / max(n_runs - 1, 1)
        R = int(round(8 * (r_max / 8) ** f))
        S = max(int(round(R * 354 / 3680)), min(8, R // 3))
        W = int(round(w_min * (w_max / w_min) ** (perm[k] / max(n_runs - 1, 1))))
        m = max(1, W // n_bins)
        net = random_network(seed * 1000 + k, S, R)
        x0 = log_uniform_counts(np.random.default_rng(seed * 1000 + k + 1), S, hi=20)
        score = x0 * np.exp(-first_order_loss(net))
        bs = int(sorted(range(S), key=lambda s: (-score[s], s))[0])
        coef = np.zeros(S)
        coef[bs] = 1.0
        out.append(WEConfig(name=f"batch{k}", net=net, x0=x0, bin_coef=coef,
                            edges=uniform_edges(0.0, 2.0 * n_bins, n_bins), m_targ=m, tau=tau,
                            n_iters=n_iters, seeds=np.array([seed * 1000 + k], np.uint64),
                            hist_species=bs, hist_lo=0, hist_hi=-1))
    return out


# --------------------------------------------------------------------------
# The batched rare-event workload: the uneven batch above, each run given a
# recycling target from pilot runs of its own.
# --------------------------------------------------------------------------
def batch_tau(events_per_walker: float, tau0: float = 0.01, target: float = 10.0,
              lo: float = 0.01, hi: float = 5.0) -> float:
    """Interval giving about `target` events per walker: tau0 scaled by
    target / (events per walker-interval measured over a pilot at tau0),
    clipped to [lo, hi] (the toggle's tau is likewise ~10 / a0)."""
    return float(np.clip(tau0 * target / max(float(events_per_walker), 1e-3), lo, hi))


def rare_target(x: np.ndarray, w: np.ndarray, tail: float = 1e-4):
    """Recycling target from a relaxed pilot ensemble (states x[n, S],
    weights w[n] summing to one): the coordinate species is the one with the
    largest weighted mean count (ties: lowest id); the recycling state A is
    the heaviest walker's state (ties: lowest slot); the threshold is the
    smallest integer t >= c_A + 2 with pilot weight P(c >= t) <= tail.
    Returns (species, x_A, threshold)."""
    x = np.asarray(x, np.int64)
    w = np.asarray(w, np.float64)
    mean = (w[:, None] * x).sum(axis=0)
    sp = int(np.flatnonzero(mean == mean.max())[0])
    xa = x[int(np.argmax(w))].astype(np.int32)
    c = x[:, sp]
    t = int(xa[sp]) + 2
    top = int(c.max()) + 1
    while t < top and w[c >= t].sum() > tail:
        t += 1
    return sp, xa, t


def rare_batch_config(base: WEConfig, tau: float, species: int, x_a: np.ndarray, thr: int,
                      n_bins: int = 16) -> WEConfig:
    """A run of the uneven batch turned into a first-passage problem: start
    and recycle at x_A, target {x_species >= thr}, n_bins equal bins on the
    species count between c_A and thr."""
    S = base.net.S
    coef = np.zeros(S, np.float64)
    coef[species] = 1.0
    ca = float(x_a[species])
    out = WEConfig(name=base.name + "_rare", net=base.net, x0=np.asarray(x_a, np.int32).copy(), bin_coef=coef,
                   edges=uniform_edges(ca, float(thr), n_bins), m_targ=base.m_targ, tau=float(tau),
                   n_iters=base.n_iters, seeds=base.seeds.copy(), recycle=True, tgt_coef=coef.copy(),
                   tgt_thr=float(thr), x_rec=np.asarray(x_a, np.int32).copy(), hist_species=species, hist_lo=0,
                   hist_hi=-1)
    out.a_thr = ca            # A region for committor labels: bin_coef . x <= c_A
    return out
