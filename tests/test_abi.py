"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/we.h declares; its host-side argument checks answer
without a device.  One GPU test drives a whole WE run through the C ABI with
plain ctypes (no binding module) and checks it against the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "we.h")
LIB = os.path.join(ROOT, "paper_1303_5986_amd", "libwe.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"WE_API\s+[\w\s\*]+?\b(we_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for core in ("we_create_network", "we_init", "we_step_intervals", "we_histogram", "we_mfpt"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libwe.so not built")
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_declares_every_symbol():
    from paper_1303_5986_amd import we
    assert sorted(we.EXPORTED) == declared_symbols()


def test_last_error_callable_without_device():
    if not os.path.exists(LIB):
        pytest.skip("libwe.so not built")
    lib = ctypes.CDLL(LIB)
    lib.we_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.we_last_error(), bytes)


def _raw_lib():
    lib = ctypes.CDLL(LIB)
    lib.we_last_error.restype = ctypes.c_char_p
    return lib


def test_host_side_argument_checks_without_device(tmp_path):
    """Invalid networks and unreadable checkpoints are refused with WE_EINVAL
    before any device call."""
    if not os.path.exists(LIB):
        pytest.skip("libwe.so not built")
    lib = _raw_lib()
    i32 = ctypes.c_int32
    A = lambda *v: (i32 * len(v))(*v)
    out = ctypes.c_void_p()
    # multiplicity 4 is beyond the mass-action orders the network accepts
    st = lib.we_create_network(1, 1, A(0, 1), A(0), A(4), A(0, 1), A(0), A(-1),
                               (ctypes.c_double * 1)(1.0), ctypes.byref(out))
    assert st == -1 and out.value is None
    assert b"multiplicity" in lib.we_last_error()
    st = lib.we_create_network(0, 1, A(0, 0), A(0), A(1), A(0, 0), A(0), A(0),
                               (ctypes.c_double * 1)(1.0), ctypes.byref(out))
    assert st == -1
    info = ctypes.create_string_buffer(128)
    assert lib.we_checkpoint_inspect(str(tmp_path / "missing.ckpt").encode(), info) == -1
    (tmp_path / "junk.ckpt").write_bytes(b"\0" * 200)
    assert lib.we_checkpoint_inspect(str(tmp_path / "junk.ckpt").encode(), info) == -1
    assert b"magic" in lib.we_last_error()


@pytest.mark.gpu
def test_c_abi_birth_death_run_matches_oracle():
    """we_create_network -> we_workspace_size -> we_init (library-allocated
    workspace, default stream) -> we_step_intervals -> we_get_walkers /
    we_histogram / we_mfpt, all through ctypes: the walkers equal the
    oracle's bit for bit and the histogram sums the weights."""
    import numpy as np
    import torch
    from oracle import oracle as orc
    from paper_1303_5986_amd import workloads as wl

    torch.cuda.init()                          # the same HIP runtime as the binding uses
    lib = _raw_lib()
    c_int, c_dbl, vp = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    ptr = lambda a: a.ctypes.data_as(vp)
    cfg = wl.birth_death_config(n_runs=2, seed0=5, n_iters=25)
    net = cfg.net
    h_net = vp()
    st = lib.we_create_network(net.S, net.R, ptr(net.reac_ptr), ptr(net.reac_species), ptr(net.reac_mult),
                               ptr(net.chg_ptr), ptr(net.chg_species), ptr(net.chg_delta), ptr(net.rate),
                               ctypes.byref(h_net))
    assert st == 0, lib.we_last_error()
    from paper_1303_5986_amd.we import _Grid, _Params
    coef = np.ascontiguousarray(cfg.bin_coef, np.float64)
    edges = np.ascontiguousarray(cfg.edges, np.float64)
    seeds = np.ascontiguousarray(cfg.seeds, np.uint64)
    x0 = np.ascontiguousarray(cfg.x0, np.int32)
    grid = _Grid(len(edges) - 1, coef.ctypes.data, edges.ctypes.data, 0, None, None)
    joint = np.zeros(1, np.int32)
    par = _Params(cfg.tau, cfg.m_targ, 2, 25, 1, seeds.ctypes.data, x0.ctypes.data, 0, None, 0.0, None,
                  0, 0, 140, 0, joint.ctypes.data, 1, 1, 0, 0, 0, 0, 0.03, 0)
    nbytes = ctypes.c_size_t()
    assert lib.we_workspace_size(h_net, ctypes.byref(grid), ctypes.byref(par), ctypes.byref(nbytes)) == 0
    h_sim = vp()
    st = lib.we_init(h_net, ctypes.byref(grid), ctypes.byref(par), None, None, ctypes.c_size_t(0),
                     ctypes.byref(h_sim))
    assert st == 0, lib.we_last_error()
    try:
        assert lib.we_step_intervals(h_sim, 25) == 0, lib.we_last_error()
        for r in range(2):
            n = c_int()
            x = np.zeros(cfg.cap, np.int32)
            w = np.zeros(cfg.cap, np.float64)
            b = np.zeros(cfg.cap, np.int32)
            o = np.zeros(cfg.cap, np.int32)
            assert lib.we_get_walkers(h_sim, r, ctypes.byref(n), ptr(x), ptr(w), ptr(b), ptr(o)) == 0
            ora = orc.OracleWE(cfg, int(cfg.seeds[r]))
            ora.step(25)
            ox, ow, ob, oo = ora.walkers()
            k = n.value
            assert k == len(ow)
            assert np.array_equal(x[:k], ox[:, 0]) and np.array_equal(w[:k], ow)
            assert np.array_equal(b[:k], ob) and np.array_equal(o[:k], oo)
            hist = np.zeros(141, np.float64)
            assert lib.we_histogram(h_sim, r, 0, 0, 140, ptr(hist)) == 0
            assert abs(hist.sum() - 1.0) < 1e-12
        mf, fm, fs = c_dbl(), c_dbl(), c_dbl()
        assert lib.we_mfpt(h_sim, 5, ctypes.byref(mf), ctypes.byref(fm), ctypes.byref(fs)) == 0
        assert fm.value == 0.0                  # no recycling target: no flux
    finally:
        lib.we_destroy.restype = None
        lib.we_destroy(h_sim)
        lib.we_destroy_network.restype = None
        lib.we_destroy_network(h_net)
