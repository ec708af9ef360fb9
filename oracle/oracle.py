"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It drives liboracle.so (we_oracle.c), a plain sequential
implementation of weighted-ensemble SSA written from the paper; see the
header of we_oracle.c for the readings it takes.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(path)
        P = C.POINTER
        L.or_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.or_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.or_u53.restype = C.c_double
        L.or_h.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32]
        L.or_h.restype = C.c_int64
        L.or_propensity.argtypes = [C.c_void_p, P(C.c_int32), C.c_int32]
        L.or_propensity.restype = C.c_double
        L.or_validate.argtypes = [C.c_void_p]
        L.or_validate.restype = C.c_int32
        L.or_ssa_interval.argtypes = [C.c_void_p, P(C.c_int32), C.c_double, C.c_uint64,
                                      C.c_uint32, C.c_uint32]
        L.or_ssa_interval.restype = C.c_int64
        L.or_tauleap_interval.argtypes = [C.c_void_p, P(C.c_int32), C.c_double, C.c_double, C.c_uint64,
                                          C.c_uint32, C.c_uint32]
        L.or_tauleap_interval.restype = C.c_int64
        L.or_ssa_first_passage.argtypes = [C.c_void_p, P(C.c_int32), C.c_double,
                                           P(C.c_double), C.c_double, C.c_uint64,
                                           C.c_uint32, P(C.c_int64)]
        L.or_ssa_first_passage.restype = C.c_double
        L.or_coord.argtypes = [C.c_int32, P(C.c_double), P(C.c_int32)]
        L.or_coord.restype = C.c_double
        L.or_bin_of.argtypes = [C.c_int32, P(C.c_double), C.c_double]
        L.or_bin_of.restype = C.c_int32
        L.or_we_iterate.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, P(C.c_int32),
                                    P(C.c_int32), P(C.c_double), P(C.c_int32),
                                    P(C.c_int32), C.c_int32, P(C.c_double), P(C.c_int64),
                                    P(C.c_int32), P(C.c_int32)]
        L.or_we_iterate.restype = C.c_int32
        L.or_resample_bin.argtypes = [C.c_int32, P(C.c_int32), P(C.c_double), C.c_int32, C.c_int32,
                                      C.c_uint64, C.c_uint32, C.c_uint32,
                                      P(C.c_int32), P(C.c_double)]
        L.or_resample_bin.restype = C.c_int32
        _LIB = L
    return _LIB


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _NetStruct(C.Structure):
    _fields_ = [("S", C.c_int32), ("R", C.c_int32),
                ("reac_ptr", C.c_void_p), ("reac_species", C.c_void_p),
                ("reac_mult", C.c_void_p), ("chg_ptr", C.c_void_p),
                ("chg_species", C.c_void_p), ("chg_delta", C.c_void_p),
                ("rate", C.c_void_p), ("hill_species", C.c_void_p), ("hill_n", C.c_void_p),
                ("hill_K", C.c_void_p)]


class _CfgStruct(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("bin_coef", C.c_void_p), ("edges", C.c_void_p),
                ("n_bins2", C.c_int32), ("bin_coef2", C.c_void_p), ("edges2", C.c_void_p),
                ("m_targ", C.c_int32), ("tau", C.c_double), ("seed", C.c_uint64),
                ("recycle", C.c_int32), ("tgt_coef", C.c_void_p), ("tgt_thr", C.c_double),
                ("x_rec", C.c_void_p), ("engine", C.c_int32), ("leap_eps", C.c_double),
                ("resample_rule", C.c_int32)]


class OracleNet:
    """Keeps the network arrays alive next to the C struct that points at them."""

    def __init__(self, net):
        self.net = net
        self._keep = [np.ascontiguousarray(a, dtype=dt) for a, dt in (
            (net.reac_ptr, np.int32), (net.reac_species, np.int32), (net.reac_mult, np.int32),
            (net.chg_ptr, np.int32), (net.chg_species, np.int32), (net.chg_delta, np.int32),
            (net.rate, np.float64))]
        k = self._keep
        hill = []
        if getattr(net, "hill_species", None) is not None:
            hill = [np.ascontiguousarray(net.hill_species, np.int32),
                    np.ascontiguousarray(net.hill_n, np.int32),
                    np.ascontiguousarray(net.hill_K, np.float64)]
            self._keep += hill
        self.s = _NetStruct(net.S, net.R, *[a.ctypes.data for a in k[:7]],
                            *([a.ctypes.data for a in hill] if hill else [None, None, None]))
        self.ptr = C.cast(C.pointer(self.s), C.c_void_p)

    def validate(self) -> int:
        return lib().or_validate(self.ptr)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def u53(hi: int, lo: int) -> float:
    return lib().or_u53(hi, lo)


def h(onet: OracleNet, x, j: int) -> int:
    xa = np.ascontiguousarray(x, dtype=np.int32)
    return lib().or_h(onet.ptr, _p(xa, C.c_int32), j)


def propensity(onet: OracleNet, x, j: int) -> float:
    xa = np.ascontiguousarray(x, dtype=np.int32)
    return lib().or_propensity(onet.ptr, _p(xa, C.c_int32), j)


def ssa_interval(onet: OracleNet, x, tau: float, seed: int, slot: int, it: int):
    xa = np.array(x, dtype=np.int32, copy=True)
    ev = lib().or_ssa_interval(onet.ptr, _p(xa, C.c_int32), tau, seed, slot, it)
    return xa, int(ev)


def tauleap_interval(onet: OracleNet, x, tau: float, eps: float, seed: int, slot: int, it: int):
    xa = np.array(x, dtype=np.int32, copy=True)
    ev = lib().or_tauleap_interval(onet.ptr, _p(xa, C.c_int32), tau, eps, seed, slot, it)
    if ev < 0:
        raise RuntimeError(f"oracle tau-leap failed: status {ev}")
    return xa, int(ev)


def first_passage(onet: OracleNet, x, T: float, coef, thr: float, seed: int, traj: int):
    xa = np.array(x, dtype=np.int32, copy=True)
    ca = np.ascontiguousarray(coef, dtype=np.float64)
    ev = C.c_int64(0)
    t = lib().or_ssa_first_passage(onet.ptr, _p(xa, C.c_int32), T, _p(ca, C.c_double),
                                   thr, seed, traj, C.byref(ev))
    return t, xa, int(ev.value)


def coord(coef, x) -> float:
    ca = np.ascontiguousarray(coef, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.int32)
    return lib().or_coord(len(ca), _p(ca, C.c_double), _p(xa, C.c_int32))


def bin_of(edges, q: float) -> int:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    return lib().or_bin_of(len(e) - 1, _p(e, C.c_double), q)


def resample_bin(slots, weights, m_targ: int, seed: int, b: int, it: int, rule: int = 0):
    s = np.ascontiguousarray(slots, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    n_out = max(m_targ, len(s), 1)
    os_ = np.zeros(n_out, np.int32)
    ow = np.zeros(n_out, np.float64)
    n = lib().or_resample_bin(len(s), _p(s, C.c_int32), _p(w, C.c_double), m_targ, rule, seed,
                              b, it, _p(os_, C.c_int32), _p(ow, C.c_double))
    return os_[:n].copy(), ow[:n].copy()


class OracleWE:
    """One WE run (one seed) of the oracle: the ensemble plus per-iteration
    outputs.  The initial ensemble is m_targ walkers at x0 with weight
    1/m_targ each, unless init_x/init_w are given."""

    def __init__(self, cfg, seed: int, init_x=None, init_w=None, rw_period: int = 0,
                 rw_reset: bool = False):
        self.cfg = cfg
        self.onet = OracleNet(cfg.net)
        st = self.onet.validate()
        if st != 0:
            raise ValueError(f"oracle: invalid network (status {st})")
        S, cap = cfg.net.S, cfg.cap
        self.seed = int(seed)
        self._arrs = dict(
            bin_coef=np.ascontiguousarray(cfg.bin_coef, np.float64),
            edges=np.ascontiguousarray(cfg.edges, np.float64),
            tgt_coef=np.ascontiguousarray(cfg.tgt_coef if cfg.tgt_coef is not None
                                          else np.zeros(S), np.float64),
            x_rec=np.ascontiguousarray(cfg.x_rec if cfg.x_rec is not None else cfg.x0, np.int32),
        )
        two_d = getattr(cfg, "edges2", None) is not None
        if two_d:
            self._arrs["bin_coef2"] = np.ascontiguousarray(cfg.bin_coef2, np.float64)
            self._arrs["edges2"] = np.ascontiguousarray(cfg.edges2, np.float64)
        a = self._arrs
        n1 = len(cfg.edges) - 1
        self.cs = _CfgStruct(n1, a["bin_coef"].ctypes.data, a["edges"].ctypes.data,
                             len(cfg.edges2) - 1 if two_d else 0,
                             a["bin_coef2"].ctypes.data if two_d else None,
                             a["edges2"].ctypes.data if two_d else None,
                             cfg.m_targ, cfg.tau, self.seed, int(bool(cfg.recycle)),
                             a["tgt_coef"].ctypes.data, float(cfg.tgt_thr), a["x_rec"].ctypes.data,
                             1 if getattr(cfg, "engine", "ssa") == "tauleap" else 0,
                             float(getattr(cfg, "leap_eps", 0.03)),
                             int(getattr(cfg, "resample_rule", 0)))
        self.cptr = C.cast(C.pointer(self.cs), C.c_void_p)
        self.x = np.zeros(cap * S, np.int32)
        self.w = np.zeros(cap, np.float64)
        self.bin = np.zeros(cap, np.int32)
        self.origin = np.full(cap, -1, np.int32)
        self.recycled = np.zeros(cap, np.int32)   # incoming slots recycled in the last step
        if init_x is None:
            n0 = cfg.m_targ
            self.x[: n0 * S] = np.tile(np.asarray(cfg.x0, np.int32), n0)
            self.w[:n0] = 1.0 / cfg.m_targ
        else:
            ix = np.asarray(init_x, np.int32).reshape(-1, S)
            n0 = ix.shape[0]
            if n0 > cap:
                raise ValueError("initial ensemble exceeds capacity")
            self.x[: n0 * S] = ix.reshape(-1)
            self.w[:n0] = np.asarray(init_w, np.float64)
        self.n = n0
        self.iter = 0
        self.flux: List[float] = []
        self.events: List[int] = []
        self.segments: List[int] = []
        # steady-state reweighting (reweight.py): every rw_period iterations
        self.rw_period = int(rw_period)
        self.rw_reset = bool(rw_reset)
        self.end_bin = np.zeros(cap, np.int32)
        self.rw_F = np.zeros((cfg.n_bins, cfg.n_bins), np.float64)
        self.rw_applied = 0
        self.rw_skipped = 0

    def step(self, n_iters: int = 1):
        L = lib()
        n = C.c_int32(self.n)
        flux = C.c_double(0.0)
        ev = C.c_int64(0)
        for _ in range(n_iters):
            n.value = self.n
            n_in = self.n
            self.segments.append(self.n)
            if self.rw_period > 0:
                start_bin = self.bin[:n_in].copy()
                start_w = self.w[:n_in].copy()
            st = L.or_we_iterate(self.onet.ptr, self.cptr, self.iter, C.byref(n),
                                 _p(self.x, C.c_int32), _p(self.w, C.c_double),
                                 _p(self.bin, C.c_int32), _p(self.origin, C.c_int32),
                                 self.cfg.cap, C.byref(flux), C.byref(ev),
                                 _p(self.recycled, C.c_int32), _p(self.end_bin, C.c_int32))
            if st != 0:
                raise RuntimeError(f"oracle WE iteration {self.iter} failed: status {st}")
            self.n = n.value
            if self.rw_period > 0:
                from . import reweight as rw
                if self.iter >= 1:
                    rw.accumulate_flux(self.rw_F, start_bin, self.end_bin[:n_in], start_w)
                if (self.iter + 1) % self.rw_period == 0:
                    if rw.reweight(self.rw_F, self.bin[:self.n], self.w[: self.n], self.cfg.n_bins):
                        self.rw_applied += 1
                    else:
                        self.rw_skipped += 1
                    if self.rw_reset:
                        self.rw_F[:] = 0.0
            self.iter += 1
            self.flux.append(flux.value)
            self.events.append(ev.value)

    # checkpoints: the ensemble after an iteration plus the series; the
    # random numbers are keyed by (seed, slot, event, iteration), so nothing
    # else is needed to continue
    _STATE = ("x", "w", "bin", "origin", "recycled", "end_bin", "rw_F")

    def save(self, path: str):
        np.savez(path, n=self.n, iter=self.iter, seed=self.seed, flux=np.array(self.flux, np.float64),
                 events=np.array(self.events, np.int64), segments=np.array(self.segments, np.int64),
                 rw=np.array([self.rw_applied, self.rw_skipped], np.int64),
                 **{k: getattr(self, k) for k in self._STATE})

    @classmethod
    def load(cls, cfg, path: str, rw_period: int = 0, rw_reset: bool = False) -> "OracleWE":
        z = np.load(path, allow_pickle=False)
        o = cls(cfg, int(z["seed"]), rw_period=rw_period, rw_reset=rw_reset)
        for k in cls._STATE:
            getattr(o, k)[...] = z[k]
        o.n = int(z["n"])
        o.iter = int(z["iter"])
        o.flux = [float(v) for v in z["flux"]]
        o.events = [int(v) for v in z["events"]]
        o.segments = [int(v) for v in z["segments"]]
        o.rw_applied, o.rw_skipped = (int(v) for v in z["rw"])
        return o

    # views of the current ensemble
    def walkers(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        S = self.cfg.net.S
        n = self.n
        return (self.x[: n * S].reshape(n, S).copy(), self.w[:n].copy(),
                self.bin[:n].copy(), self.origin[:n].copy())

    def child_recycled(self) -> np.ndarray:
        """For each walker of the current ensemble: 1 if its parent reached B
        (and was recycled) in the last iteration."""
        return self.recycled[self.origin[: self.n]].copy()

    def histogram(self, species: int, lo: int, hi: int) -> np.ndarray:
        """P(x_species = k) for k in [lo, hi] from the current ensemble (walker
        weights summed in slot order)."""
        S = self.cfg.net.S
        out = np.zeros(hi - lo + 1, np.float64)
        xs = self.x[: self.n * S].reshape(self.n, S)[:, species]
        for k in range(self.n):
            v = int(xs[k])
            if lo <= v <= hi:
                out[v - lo] += self.w[k]
        return out


def mfpt_from_flux(flux_runs: np.ndarray, tau: float, discard: int):
    """MFPT = 1 / steady-state flux (Eq. mfpt).  flux_runs[r, i] is the weight
    recycled in iteration i of run r; per run the flux is its mean after
    `discard` iterations divided by tau; runs are independent samples
    (Sec. III.C treats replica means as independent points)."""
    f = np.asarray(flux_runs, np.float64)[:, discard:]
    per_run = f.mean(axis=1) / tau
    mean = per_run.mean()
    sem = per_run.std(ddof=1) / np.sqrt(len(per_run)) if len(per_run) > 1 else float("nan")
    return 1.0 / mean if mean > 0 else float("inf"), mean, sem
