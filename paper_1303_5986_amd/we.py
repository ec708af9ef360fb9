"""Python binding of libwe.so (the C ABI in include/we.h).

Argument marshalling only: every step of the WE iteration runs in the HIP
kernels of libwe.so.  PyTorch supplies the device workspace and the stream.
There is no CPU fallback: if libwe.so is missing or no HIP device is
present, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwe.so")

WE_OK, WE_EINVAL, WE_ENOMEM, WE_EDEVICE, WE_ECAPACITY, WE_EOVERFLOW, WE_ESTATE = 0, -1, -2, -3, -4, -5, -6
WE_KERNEL_AUTO, WE_KERNEL_LANE, WE_KERNEL_WAVE, WE_KERNEL_GROUP = 0, 1, 2, 3
WE_COUNT_MAX = 131071

_STATUS = {WE_EINVAL: "EINVAL", WE_ENOMEM: "ENOMEM", WE_EDEVICE: "EDEVICE",
           WE_ECAPACITY: "ECAPACITY", WE_EOVERFLOW: "EOVERFLOW", WE_ESTATE: "ESTATE"}

EXPORTED = [
    "we_create_network", "we_destroy_network", "we_set_hill", "we_workspace_size", "we_init",
    "we_set_ensemble",
    "we_step_intervals", "we_graph_capture", "we_graph_replay", "we_synchronize", "we_get_walkers",
    "we_histogram", "we_histogram_accum", "we_joint_histogram", "we_flux", "we_mfpt",
    "we_counters", "we_events_series", "we_rw_flux_matrix", "we_rw_counts", "we_profile",
    "we_profile_read",
    "we_train_committor", "we_use_committor_bins", "we_committor_eval", "we_committor_state",
    "we_record_labels", "we_get_record", "we_mlp_loss_grad", "we_mlp_loss_grad_noalloc", "we_adam_step",
    "we_batch_create", "we_batch_step", "we_batch_graph_capture", "we_batch_graph_replay",
    "we_batch_sim", "we_batch_info", "we_batch_destroy", "we_measure_peaks", "we_walker_events",
    "we_set_bins", "we_save", "we_checkpoint_inspect", "we_load", "we_propagation_kernel",
    "we_destroy", "we_last_error",
]

N_HIDDEN = 64


def n_params(n_in: int) -> int:
    """Parameters of the committor model n_in -> 64 -> 64 -> 1."""
    return N_HIDDEN * n_in + N_HIDDEN + N_HIDDEN * N_HIDDEN + N_HIDDEN + N_HIDDEN + 1


class WEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Grid(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("coef", C.c_void_p), ("edges", C.c_void_p),
                ("n_bins2", C.c_int32), ("coef2", C.c_void_p), ("edges2", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("m_targ", C.c_int32), ("n_runs", C.c_int32),
                ("max_iters", C.c_int32), ("kernel", C.c_int32), ("seeds", C.c_void_p),
                ("x0", C.c_void_p), ("recycle", C.c_int32), ("tgt_coef", C.c_void_p),
                ("tgt_thr", C.c_double), ("x_rec", C.c_void_p), ("hist_species", C.c_int32),
                ("hist_lo", C.c_int32), ("hist_hi", C.c_int32), ("n_joint", C.c_int32),
                ("joint_species", C.c_void_p), ("joint_bins", C.c_int32), ("joint_width", C.c_int32),
                ("record_iters", C.c_int32), ("rw_period", C.c_int32), ("rw_reset", C.c_int32),
                ("engine", C.c_int32), ("leap_eps", C.c_double), ("resample_rule", C.c_int32),
                ("walkers_per_wave", C.c_int32)]


class _Peaks(C.Structure):
    _fields_ = [("hbm_gbs", C.c_double), ("lds_tbs", C.c_double), ("fp64_tflops", C.c_double),
                ("int32_tops", C.c_double), ("compute_units", C.c_int32)]


class _Bins(C.Structure):
    _fields_ = [("kind", C.c_int32), ("grid", C.c_void_p), ("qedges", C.c_void_p)]


class _CheckpointInfo(C.Structure):
    _fields_ = [("version", C.c_int32), ("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("n_runs", C.c_int32), ("n_bins", C.c_int32), ("m_targ", C.c_int32),
                ("max_iters", C.c_int32), ("iteration", C.c_int32), ("hist_lo", C.c_int32),
                ("hist_hi", C.c_int32), ("n_joint", C.c_int32), ("joint_bins", C.c_int32),
                ("kernel", C.c_int32), ("tau", C.c_double), ("workspace_bytes", C.c_uint64)]


WE_BINS_GRID, WE_BINS_LEARNED = 0, 1


class _TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("a_coef", C.c_void_p), ("a_thr", C.c_double), ("seed", C.c_uint64),
                ("edge_mode", C.c_int32)]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libwe.so and declare its signatures.  Raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libwe.so not built ({path}); run __graft_entry__.build()")
    # torch ships its own libamdhip64 with the same soname as ROCm's: load and
    # initialise it first so libwe.so binds to that one runtime, not a second.
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: libwe.so runs on MI355X only")
    torch.cuda.init()
    L = C.CDLL(path)
    P, vp, i32, i64, f64 = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.we_create_network.argtypes = [i32, i32] + [vp] * 7 + [P(vp)]
    L.we_set_hill.argtypes = [vp, i32, i32, i32, f64]
    L.we_destroy_network.argtypes = [vp]
    L.we_destroy_network.restype = None
    L.we_workspace_size.argtypes = [vp, vp, vp, P(C.c_size_t)]
    L.we_init.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, P(vp)]
    L.we_set_ensemble.argtypes = [vp, i32, i32, vp, vp]
    L.we_step_intervals.argtypes = [vp, i32]
    L.we_graph_capture.argtypes = [vp, i32]
    L.we_graph_replay.argtypes = [vp, i32]
    L.we_synchronize.argtypes = [vp]
    L.we_get_walkers.argtypes = [vp, i32, P(i32), vp, vp, vp, vp]
    L.we_histogram.argtypes = [vp, i32, i32, i32, i32, vp]
    L.we_histogram_accum.argtypes = [vp, vp, P(i32)]
    L.we_joint_histogram.argtypes = [vp, vp]
    L.we_flux.argtypes = [vp, i32, i32, i32, vp]
    L.we_mfpt.argtypes = [vp, i32, P(f64), P(f64), P(f64)]
    L.we_counters.argtypes = [vp, P(i64), P(i64), P(i32)]
    L.we_events_series.argtypes = [vp, i32, i32, vp]
    L.we_rw_flux_matrix.argtypes = [vp, i32, vp]
    L.we_rw_counts.argtypes = [vp, i32, P(i32), P(i32)]
    L.we_profile.argtypes = [vp, i32]
    L.we_profile_read.argtypes = [vp, P(f64), P(f64), P(f64), P(i64)]
    L.we_train_committor.argtypes = [vp, vp, vp, P(i32)]
    L.we_use_committor_bins.argtypes = [vp, i32]
    L.we_committor_eval.argtypes = [vp, i32, vp, vp]
    L.we_committor_state.argtypes = [vp, vp, vp, vp, P(i32)]
    L.we_record_labels.argtypes = [vp, vp, f64, vp, P(i32)]
    L.we_get_record.argtypes = [vp, i32, vp, vp, vp, vp]
    L.we_mlp_loss_grad.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp]
    L.we_mlp_loss_grad_noalloc.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp]
    L.we_adam_step.argtypes = [i32, vp, vp, vp, vp, C.c_float, i32]
    L.we_batch_create.argtypes = [i32, vp, vp, vp, vp, i32, C.c_char_p, P(vp)]
    L.we_batch_step.argtypes = [vp, i32]
    L.we_batch_graph_capture.argtypes = [vp, i32]
    L.we_batch_graph_replay.argtypes = [vp, i32]
    L.we_batch_sim.argtypes = [vp, i32]
    L.we_batch_sim.restype = vp
    L.we_batch_info.argtypes = [vp, P(i32), vp, vp]
    L.we_measure_peaks.argtypes = [vp, vp]
    L.we_walker_events.argtypes = [vp, i32, P(i32), vp]
    L.we_batch_destroy.argtypes = [vp]
    L.we_batch_destroy.restype = None
    L.we_set_bins.argtypes = [vp, vp]
    L.we_propagation_kernel.argtypes = [vp]
    L.we_propagation_kernel.restype = C.c_char_p
    L.we_save.argtypes = [vp, C.c_char_p]
    L.we_checkpoint_inspect.argtypes = [C.c_char_p, vp]
    L.we_load.argtypes = [vp, C.c_char_p, vp, vp, C.c_size_t, P(vp)]
    L.we_destroy.argtypes = [vp]
    L.we_destroy.restype = None
    L.we_last_error.restype = C.c_char_p
    for name in EXPORTED:
        fn = getattr(L, name)
        if name not in ("we_destroy", "we_destroy_network", "we_last_error", "we_batch_sim",
                        "we_batch_destroy", "we_propagation_kernel"):
            fn.restype = C.c_int
    _LIB = L
    return L


def _check(st: int):
    if st != WE_OK:
        raise WEError(st, load_library().we_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Network:
    """A compiled reaction network on the device (we_create_network)."""

    def __init__(self, net):
        L = load_library()
        self.net = net
        self.S, self.R = int(net.S), int(net.R)
        arrs = [np.ascontiguousarray(getattr(net, k), dtype=np.int32) for k in
                ("reac_ptr", "reac_species", "reac_mult", "chg_ptr", "chg_species", "chg_delta")]
        rate = np.ascontiguousarray(net.rate, dtype=np.float64)
        h = C.c_void_p()
        _check(L.we_create_network(self.S, self.R, *[_ptr(a) for a in arrs], _ptr(rate),
                                   C.byref(h)))
        self.handle = h
        if getattr(net, "hill_species", None) is not None:
            for j in range(self.R):
                if int(net.hill_species[j]) >= 0:
                    _check(L.we_set_hill(self.handle, j, int(net.hill_species[j]), int(net.hill_n[j]),
                                         float(net.hill_K[j])))

    def close(self):
        if getattr(self, "handle", None):
            load_library().we_destroy_network(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim:
    """n_runs independent WE runs of one network on the current HIP device.

    The workspace is a torch uint8 tensor; kernels run on torch's current
    stream of that device."""

    def __init__(self, network: Network, bin_coef, edges, *, tau: float, m_targ: int,
                 seeds: Sequence[int], x0, max_iters: int, kernel: int = WE_KERNEL_AUTO,
                 recycle: bool = False, tgt_coef=None, tgt_thr: float = 0.0, x_rec=None,
                 hist_species: int = 0, hist_lo: int = 0, hist_hi: int = -1,
                 joint_species: Sequence[int] = (), joint_bins: int = 16, joint_width: int = 64,
                 record_iters: int = 0, rw_period: int = 0, rw_reset: bool = False,
                 bin_coef2=None, edges2=None, engine: str = "ssa", leap_eps: float = 0.03,
                 resample_rule: int = 0, walkers_per_wave: int = 0, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: libwe.so runs on MI355X only")
        L = load_library()
        self.network = network
        S = network.S
        self._keep = dict(
            coef=np.ascontiguousarray(bin_coef, np.float64),
            edges=np.ascontiguousarray(edges, np.float64),
            seeds=np.ascontiguousarray(seeds, np.uint64),
            x0=np.ascontiguousarray(x0, np.int32),
            tgt=None if tgt_coef is None else np.ascontiguousarray(tgt_coef, np.float64),
            xrec=None if x_rec is None else np.ascontiguousarray(x_rec, np.int32),
            joint=np.ascontiguousarray(list(joint_species) or [0], np.int32),
            coef2=None if bin_coef2 is None else np.ascontiguousarray(bin_coef2, np.float64),
            edges2=None if edges2 is None else np.ascontiguousarray(edges2, np.float64),
        )
        k = self._keep
        if k["coef"].shape != (S,) or k["x0"].shape != (S,):
            raise ValueError("bin_coef and x0 need one entry per species")
        n2 = 0 if k["edges2"] is None else len(k["edges2"]) - 1
        self.n_bins = (len(k["edges"]) - 1) * max(n2, 1)
        self.n_runs = len(k["seeds"])
        self.m_targ = int(m_targ)
        self.cap = self.m_targ * self.n_bins
        self.S = S
        self.tau = float(tau)
        self.grid = _Grid(len(k["edges"]) - 1, k["coef"].ctypes.data, k["edges"].ctypes.data,
                          n2, _ptr(k["coef2"]), _ptr(k["edges2"]))
        self.params = _Params(float(tau), int(m_targ), self.n_runs, int(max_iters), int(kernel),
                              k["seeds"].ctypes.data, k["x0"].ctypes.data, int(bool(recycle)),
                              _ptr(k["tgt"]), float(tgt_thr), _ptr(k["xrec"]),
                              int(hist_species), int(hist_lo), int(hist_hi),
                              len(joint_species), k["joint"].ctypes.data, int(joint_bins),
                              int(joint_width), int(record_iters), int(rw_period), int(bool(rw_reset)),
                              {"ssa": 0, "tauleap": 1}[engine], float(leap_eps), int(resample_rule),
                              int(walkers_per_wave))
        self.n_joint = len(joint_species)
        self.joint_cells = int(joint_bins) ** self.n_joint if self.n_joint else 0
        self.nh = hist_hi - hist_lo + 1 if hist_hi >= hist_lo else 0
        nbytes = C.c_size_t(0)
        _check(L.we_workspace_size(network.handle, C.byref(self.grid), C.byref(self.params),
                                   C.byref(nbytes)))
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        with torch.cuda.device(dev):
            self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
            self.stream = torch.cuda.current_stream(dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        h = C.c_void_p()
        _check(L.we_init(network.handle, C.byref(self.grid), C.byref(self.params),
                         C.c_void_p(self.stream.cuda_stream), C.c_void_p(aligned),
                         C.c_size_t(int(nbytes.value)), C.byref(h)))
        self.handle = h

    def propagation_kernel(self) -> str:
        """Name of the propagation kernel this sim's steps launch."""
        return load_library().we_propagation_kernel(self.handle).decode()

    # ------------------------------------------------------------ checkpoints, bins
    def save(self, path: str):
        """Write a checkpoint of every run at the current iteration."""
        _check(load_library().we_save(self.handle, os.fspath(path).encode()))

    @classmethod
    def load(cls, network: "Network", path: str, device=None) -> "Sim":
        """A sim rebuilt from a checkpoint saved on `network`."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: libwe.so runs on MI355X only")
        L = load_library()
        info = checkpoint_info(path)
        self = cls.__new__(cls)
        self.network = network
        self.S = info.n_species
        self.n_bins = info.n_bins
        self.n_runs = info.n_runs
        self.m_targ = info.m_targ
        self.cap = self.m_targ * self.n_bins
        self.tau = info.tau
        self.n_joint = info.n_joint
        self.joint_cells = int(info.joint_bins) ** self.n_joint if self.n_joint else 0
        self.nh = info.hist_hi - info.hist_lo + 1 if info.hist_hi >= info.hist_lo else 0
        self._keep = {}
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        nbytes = int(info.workspace_bytes)
        with torch.cuda.device(dev):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            self.stream = torch.cuda.current_stream(dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        h = C.c_void_p()
        _check(L.we_load(network.handle, os.fspath(path).encode(), C.c_void_p(self.stream.cuda_stream),
                         C.c_void_p(aligned), C.c_size_t(nbytes), C.byref(h)))
        self.handle = h
        return self

    def set_grid_bins(self, bin_coef=None, edges=None, bin_coef2=None, edges2=None):
        """Bin on a new grid with the same number of bins per axis, or (no
        arguments) on the sim's grid again after learned bins."""
        if edges is None:
            _check(load_library().we_set_bins(self.handle, C.byref(_Bins(WE_BINS_GRID, None, None))))
            return
        k = dict(coef=np.ascontiguousarray(bin_coef, np.float64), edges=np.ascontiguousarray(edges, np.float64),
                 coef2=None if bin_coef2 is None else np.ascontiguousarray(bin_coef2, np.float64),
                 edges2=None if edges2 is None else np.ascontiguousarray(edges2, np.float64))
        n2 = 0 if k["edges2"] is None else len(k["edges2"]) - 1
        g = _Grid(len(k["edges"]) - 1, k["coef"].ctypes.data, k["edges"].ctypes.data, n2,
                  _ptr(k["coef2"]), _ptr(k["edges2"]))
        _check(load_library().we_set_bins(self.handle, C.byref(_Bins(WE_BINS_GRID, C.addressof(g), None))))

    def set_learned_bins(self, qedges=None):
        """Bin on the trained committor; qedges (n_bins + 1 logit edges)
        replaces the edges computed at training."""
        q = None if qedges is None else np.ascontiguousarray(qedges, np.float64)
        if q is not None and len(q) != self.n_bins + 1:
            raise ValueError(f"need {self.n_bins + 1} logit edges, got {len(q)}")
        _check(load_library().we_set_bins(self.handle, C.byref(_Bins(WE_BINS_LEARNED, None, _ptr(q)))))

    # ------------------------------------------------------------ stepping
    def set_ensemble(self, run: int, x, w):
        x = np.ascontiguousarray(x, np.int32).reshape(-1)
        w = np.ascontiguousarray(w, np.float64)
        _check(load_library().we_set_ensemble(self.handle, run, len(w), _ptr(x), _ptr(w)))

    def step(self, n: int = 1):
        _check(load_library().we_step_intervals(self.handle, int(n)))

    def graph_capture(self, n: int):
        """Capture n (even) iterations as a HIP graph."""
        _check(load_library().we_graph_capture(self.handle, int(n)))

    def graph_replay(self, times: int = 1):
        _check(load_library().we_graph_replay(self.handle, int(times)))

    def synchronize(self):
        _check(load_library().we_synchronize(self.handle))

    # ------------------------------------------------------------ outputs
    def walkers(self, run: int):
        n = C.c_int32(0)
        x = np.zeros(self.cap * self.S, np.int32)
        w = np.zeros(self.cap, np.float64)
        b = np.zeros(self.cap, np.int32)
        o = np.zeros(self.cap, np.int32)
        _check(load_library().we_get_walkers(self.handle, run, C.byref(n), _ptr(x), _ptr(w),
                                             _ptr(b), _ptr(o)))
        m = n.value
        return x[: m * self.S].reshape(m, self.S), w[:m], b[:m], o[:m]

    def histogram(self, run: int, species: int, lo: int, hi: int) -> np.ndarray:
        out = np.zeros(hi - lo + 1, np.float64)
        _check(load_library().we_histogram(self.handle, run, species, lo, hi, _ptr(out)))
        return out

    def histogram_accum(self):
        out = np.zeros(self.n_runs * self.nh, np.float64)
        n = C.c_int32(0)
        _check(load_library().we_histogram_accum(self.handle, _ptr(out), C.byref(n)))
        return out.reshape(self.n_runs, self.nh), n.value

    def joint_histogram(self) -> np.ndarray:
        out = np.zeros(self.n_runs * self.joint_cells, np.float64)
        _check(load_library().we_joint_histogram(self.handle, _ptr(out)))
        return out.reshape(self.n_runs, self.joint_cells)

    def flux(self, run: int, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = self.iterations - first
        out = np.zeros(count, np.float64)
        _check(load_library().we_flux(self.handle, run, first, count, _ptr(out)))
        return out

    def mfpt(self, discard: int):
        m, f, e = C.c_double(), C.c_double(), C.c_double()
        _check(load_library().we_mfpt(self.handle, discard, C.byref(m), C.byref(f), C.byref(e)))
        return m.value, f.value, e.value

    def rw_flux_matrix(self, run: int) -> np.ndarray:
        """Reweighting's flux matrix of run `run`: F[i, j], weight moved
        from bin j into bin i."""
        out = np.zeros(self.n_bins * self.n_bins, np.float64)
        _check(load_library().we_rw_flux_matrix(self.handle, run, _ptr(out)))
        return out.reshape(self.n_bins, self.n_bins)

    def rw_counts(self, run: int):
        """(applied, skipped) reweighting events of run `run`."""
        ap, sk = C.c_int32(), C.c_int32()
        _check(load_library().we_rw_counts(self.handle, run, C.byref(ap), C.byref(sk)))
        return ap.value, sk.value

    def counters(self):
        ev, sg, it = C.c_int64(), C.c_int64(), C.c_int32()
        _check(load_library().we_counters(self.handle, C.byref(ev), C.byref(sg), C.byref(it)))
        return ev.value, sg.value, it.value

    def walker_events(self, run: int) -> np.ndarray:
        """Reactions fired by each walker of `run` in the last interval."""
        out = np.zeros(self.cap, np.uint32)
        n = C.c_int32(0)
        _check(load_library().we_walker_events(self.handle, int(run), C.byref(n), _ptr(out)))
        return out[: n.value]

    def events_series(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = self.iterations - first
        out = np.zeros(count, np.int64)
        _check(load_library().we_events_series(self.handle, first, count, _ptr(out)))
        return out

    # ------------------------------------------------------------ learned bins
    def train_committor(self, a_coef, a_thr: float, steps: int = 2000, batch: int = 1024,
                        lr: float = 1e-3, seed: int = 1, edge_mode: int = 0):
        """Train the committor on the recorded iterations; returns
        (per-step loss, number of training states)."""
        a = np.ascontiguousarray(a_coef, np.float64)
        tp = _TrainParams(int(steps), int(batch), float(lr), a.ctypes.data, float(a_thr), int(seed),
                          int(edge_mode))
        loss = np.zeros(max(int(steps), 1), np.float32)
        n = C.c_int32(0)
        _check(load_library().we_train_committor(self.handle, C.byref(tp), _ptr(loss), C.byref(n)))
        return loss[:steps], n.value

    def use_committor_bins(self, enable: bool = True):
        _check(load_library().we_use_committor_bins(self.handle, int(bool(enable))))

    def committor(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, np.int32).reshape(-1, self.S)
        q = np.zeros(len(x), np.float32)
        _check(load_library().we_committor_eval(self.handle, len(x), _ptr(x), _ptr(q)))
        return q

    def committor_state(self):
        npar = n_params(self.S)
        p = np.zeros(npar, np.float32)
        f = np.zeros(2 * self.S, np.float32)
        e = np.zeros(self.n_bins + 1, np.float64)
        n = C.c_int32(0)
        _check(load_library().we_committor_state(self.handle, _ptr(p), _ptr(f), _ptr(e), C.byref(n)))
        return p, f, e

    def record_labels(self, a_coef, a_thr: float, n_rec: int):
        a = np.ascontiguousarray(a_coef, np.float64)
        out = np.zeros(2 * n_rec * self.n_runs * self.cap, np.uint32)
        n = C.c_int32(0)
        _check(load_library().we_record_labels(self.handle, _ptr(a), float(a_thr), _ptr(out),
                                               C.byref(n)))
        return out.reshape(n_rec, self.n_runs, self.cap, 2)[: n.value]

    def record(self, i: int):
        W = self.n_runs * self.cap
        n = np.zeros(self.n_runs, np.int32)
        x = np.zeros(W * self.S, np.int32)
        o = np.zeros(W, np.int32)
        r = np.zeros(W, np.uint8)
        _check(load_library().we_get_record(self.handle, i, _ptr(n), _ptr(x), _ptr(o), _ptr(r)))
        return n, x.reshape(self.n_runs, self.cap, self.S), o.reshape(self.n_runs, self.cap), \
            r.reshape(self.n_runs, self.cap)

    def profile(self, enable: bool = True):
        _check(load_library().we_profile(self.handle, int(bool(enable))))

    def profile_read(self):
        """(ms in SSA kernels, ms in resample kernels, ms in observe kernels,
        iterations covered), from HIP events on the sim's stream."""
        a, b, c, n = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        _check(load_library().we_profile_read(self.handle, C.byref(a), C.byref(b), C.byref(c),
                                              C.byref(n)))
        return a.value, b.value, c.value, n.value

    @property
    def iterations(self) -> int:
        return self.counters()[2]

    def close(self):
        if getattr(self, "handle", None):
            load_library().we_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sim_from_config(cfg, *, kernel: int = WE_KERNEL_AUTO, max_iters: Optional[int] = None,
                    network: Optional[Network] = None, joint: bool = False,
                    record_iters: int = 0, rw_period: int = 0, rw_reset: bool = False,
                    walkers_per_wave: int = 0) -> Sim:
    """Build a Sim from a workloads.WEConfig."""
    net = network if network is not None else Network(cfg.net)
    return Sim(net, cfg.bin_coef, cfg.edges, tau=cfg.tau, m_targ=cfg.m_targ, seeds=cfg.seeds,
               x0=cfg.x0, max_iters=max_iters if max_iters is not None else cfg.n_iters,
               kernel=kernel, recycle=cfg.recycle, tgt_coef=cfg.tgt_coef, tgt_thr=cfg.tgt_thr,
               x_rec=cfg.x_rec, hist_species=cfg.hist_species, hist_lo=cfg.hist_lo,
               hist_hi=cfg.hist_hi,
               joint_species=getattr(cfg, "joint_species", ()) if joint else (),
               record_iters=record_iters, rw_period=rw_period, rw_reset=rw_reset,
               bin_coef2=getattr(cfg, "bin_coef2", None), edges2=getattr(cfg, "edges2", None),
               engine=getattr(cfg, "engine", "ssa"), leap_eps=getattr(cfg, "leap_eps", 0.03),
               resample_rule=getattr(cfg, "resample_rule", 0), walkers_per_wave=walkers_per_wave)


def mlp_loss_grad(n_in: int, params, feat, x, y):
    """Loss and gradient of the committor model on one minibatch, computed by
    the library's training kernels (default stream)."""
    p = np.ascontiguousarray(params, np.float32)
    f = np.ascontiguousarray(feat, np.float32)
    xx = np.ascontiguousarray(x, np.int32).reshape(-1)
    yy = np.ascontiguousarray(y, np.float32)
    g = np.zeros(n_params(n_in), np.float32)
    loss = np.zeros(1, np.float32)
    _check(load_library().we_mlp_loss_grad(n_in, _ptr(p), _ptr(f), len(yy), _ptr(xx), _ptr(yy),
                                           _ptr(loss), _ptr(g)))
    return float(loss[0]), g


def mlp_loss_grad_noalloc(n_in: int, params, feat, x, y, loss, grad, stream=None):
    """we_mlp_loss_grad_noalloc on torch device tensors (float32 params[n_params],
    feat[2*n_in], y[batch], loss[1], grad[n_params]; int32 x[batch, n_in]),
    launched on `stream` (default: torch's current stream).  Asynchronous."""
    import torch
    for t in (params, feat, x, y, loss, grad):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("mlp_loss_grad_noalloc needs contiguous device tensors")
    st = stream if stream is not None else torch.cuda.current_stream()
    batch = int(y.numel())
    vp = C.c_void_p
    _check(load_library().we_mlp_loss_grad_noalloc(
        int(n_in), vp(params.data_ptr()), vp(feat.data_ptr()), batch, vp(x.data_ptr()),
        vp(y.data_ptr()), vp(loss.data_ptr()), vp(grad.data_ptr()), vp(st.cuda_stream)))


def checkpoint_info(path: str) -> _CheckpointInfo:
    """Sizes recorded in a checkpoint file (reads its header only)."""
    info = _CheckpointInfo()
    _check(load_library().we_checkpoint_inspect(os.fspath(path).encode(), C.byref(info)))
    return info


def adam_step(params, m, v, grad, lr: float, t: int):
    p = np.array(params, np.float32)
    mm = np.array(m, np.float32)
    vv = np.array(v, np.float32)
    g = np.ascontiguousarray(grad, np.float32)
    _check(load_library().we_adam_step(len(p), _ptr(p), _ptr(mm), _ptr(vv), _ptr(g), float(lr),
                                       int(t)))
    return p, mm, vv


class _MemberSim(Sim):
    """A member of a Batch: the getters of Sim on a handle the batch owns."""

    def __init__(self, batch, i, cfg):
        self.handle = C.c_void_p(load_library().we_batch_sim(batch.handle, i))
        self.network = batch.networks[i]
        self.S = cfg.net.S
        self.n_bins = cfg.n_bins
        self.n_runs = len(cfg.seeds)
        self.m_targ = cfg.m_targ
        self.cap = cfg.m_targ * cfg.n_bins
        self.tau = cfg.tau
        self.nh = cfg.hist_hi - cfg.hist_lo + 1 if cfg.hist_hi >= cfg.hist_lo else 0
        self.n_joint = 0
        self.joint_cells = 0
        self._owner = batch

    def close(self):
        self.handle = None


class Batch:
    """Independent WE runs of different networks stepped together: one
    persistent propagation launch per kernel variant (we_batch_create)."""

    def __init__(self, cfgs, *, max_iters: int, autotune_iters: int = 0,
                 cache_path: Optional[str] = None, kernels=None, record_iters: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: libwe.so runs on MI355X only")
        L = load_library()
        n = len(cfgs)
        self.cfgs = cfgs
        self.networks = [Network(c.net) for c in cfgs]
        self._keep = []
        grids = (_Grid * n)()
        params = (_Params * n)()
        for i, c in enumerate(cfgs):
            k = dict(coef=np.ascontiguousarray(c.bin_coef, np.float64),
                     edges=np.ascontiguousarray(c.edges, np.float64),
                     seeds=np.ascontiguousarray(c.seeds, np.uint64),
                     x0=np.ascontiguousarray(c.x0, np.int32),
                     tgt=None if c.tgt_coef is None else np.ascontiguousarray(c.tgt_coef, np.float64),
                     xrec=None if c.x_rec is None else np.ascontiguousarray(c.x_rec, np.int32),
                     joint=np.zeros(1, np.int32))
            self._keep.append(k)
            e2 = getattr(c, "edges2", None)
            if e2 is not None:
                k["coef2"] = np.ascontiguousarray(c.bin_coef2, np.float64)
                k["edges2"] = np.ascontiguousarray(e2, np.float64)
            grids[i] = _Grid(len(k["edges"]) - 1, k["coef"].ctypes.data, k["edges"].ctypes.data,
                             0 if e2 is None else len(e2) - 1, _ptr(k.get("coef2")), _ptr(k.get("edges2")))
            kern = WE_KERNEL_AUTO if kernels is None else kernels[i]
            kern, wpw = (int(kern[0]), int(kern[1])) if isinstance(kern, tuple) else (int(kern), 0)
            params[i] = _Params(float(c.tau), int(c.m_targ), len(k["seeds"]), int(max_iters), kern,
                                k["seeds"].ctypes.data, k["x0"].ctypes.data, int(bool(c.recycle)),
                                _ptr(k["tgt"]), float(c.tgt_thr), _ptr(k["xrec"]),
                                int(c.hist_species), int(c.hist_lo), int(c.hist_hi),
                                0, k["joint"].ctypes.data, 1, 1, int(record_iters), 0, 0,
                                {"ssa": 0, "tauleap": 1}[getattr(c, "engine", "ssa")],
                                float(getattr(c, "leap_eps", 0.03)),
                                int(getattr(c, "resample_rule", 0)), wpw)
        nets = (C.c_void_p * n)(*[net.handle.value for net in self.networks])
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        _check(L.we_batch_create(n, nets, grids, params, C.c_void_p(self.stream.cuda_stream),
                                 int(autotune_iters),
                                 None if cache_path is None else cache_path.encode(), C.byref(h)))
        self.handle = h
        self.members = [_MemberSim(self, i, c) for i, c in enumerate(cfgs)]

    def step(self, n: int = 1):
        _check(load_library().we_batch_step(self.handle, int(n)))

    def graph_capture(self, n: int):
        _check(load_library().we_batch_graph_capture(self.handle, int(n)))

    def graph_replay(self, times: int = 1):
        _check(load_library().we_batch_graph_replay(self.handle, int(times)))

    def kernels(self):
        k = np.zeros(len(self.cfgs), np.int32)
        n = C.c_int32()
        _check(load_library().we_batch_info(self.handle, C.byref(n), _ptr(k), None))
        return k

    def walkers_per_wave(self):
        """Walkers per wave of every member's kernel: 64 lane, 2..32 group, 1 wave."""
        w = np.zeros(len(self.cfgs), np.int32)
        n = C.c_int32()
        _check(load_library().we_batch_info(self.handle, C.byref(n), None, _ptr(w)))
        return w

    def synchronize(self):
        for m in self.members:
            m.synchronize()

    def close(self):
        if getattr(self, "handle", None):
            load_library().we_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks() -> dict:
    """we_measure_peaks on torch's current stream: measured HBM (GB/s), LDS
    (TB/s), FP64 (TFLOP/s) and int32 lane-operation (10^12/s) ceilings."""
    import torch
    pk = _Peaks()
    _check(load_library().we_measure_peaks(C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(pk)))
    return {"hbm_gbs": pk.hbm_gbs, "lds_tbs": pk.lds_tbs, "fp64_tflops": pk.fp64_tflops,
            "int32_tops": pk.int32_tops, "compute_units": pk.compute_units}


def autotune(cfg, iters: int = 3, cache_path: Optional[str] = None):
    """(kernel, walkers_per_wave) that the batch autotuner picks for one
    configuration: every kernel its network fits (lane, group with 32..2
    walkers per wave, wave) timed on one interval of a pilot sim of the
    configuration's shape with every slot filled at x0 (best of `iters`
    pilots); walkers_per_wave is 0 unless the group kernel wins."""
    b = Batch([cfg], max_iters=2, autotune_iters=int(iters), cache_path=cache_path)
    try:
        k, w = int(b.kernels()[0]), int(b.walkers_per_wave()[0])
    finally:
        b.close()
    return k, (w if k == WE_KERNEL_GROUP else 0)

