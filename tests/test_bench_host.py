"""Host-side checks of bench.py's bookkeeping (CPU only): the algorithmic
operation count that prices an event on the ALU roofline, the source digest
that ties a committed HBM-traffic record to the kernel code it was measured
on, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1303_5986_amd import workloads as wl  # noqa: E402


def test_ops_per_event_schlogl_by_hand():
    """Philox 60 (20 products, 40 xors) + uniforms 10 + waiting time 5 +
    target/time 2, and per reaction 5 + f_j: A+2X->3X (C(x,2): 3), 3X->A+2X (C(x,3): 6), B->X (0),
    X->B (0), so 4 x 5 + 9 = 29; one changed species + 2 bound checks."""
    assert bench.alg_ops_per_event(wl.schlogl()) == 60 + 10 + 5 + 2 + 29 + 1 + 2 == 109


def test_ops_per_event_two_species_reaction():
    """A + B -> C adds the two-species product (1) to 5; mean changed
    species 3."""
    net = wl.Network.from_reactions(["A", "B", "C"], [({"A": 1, "B": 1}, {"C": 1}, 1.0)])
    assert bench.alg_ops_per_event(net) == 60 + 10 + 5 + 2 + 6 + 3 + 2


def test_source_digest_ignores_comments_only(tmp_path):
    a = tmp_path / "a.h"
    a.write_text("int f(int x) {  // first\n    return x + 1; /* one */\n}\n")
    d0 = bench.source_digest([str(a)])
    a.write_text("// a header comment\nint f(int x) {\n  return x + 1;   // reworded\n}\n")
    assert bench.source_digest([str(a)]) == d0
    a.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.source_digest([str(a)]) != d0


def test_traffic_record_needs_matching_digest(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_traffic.json").write_text('{"source_digest": "abc", "bytes_per_launch": 123.0}')
    assert bench.traffic_from_profiles("k", "abc") == 123.0
    assert bench.traffic_from_profiles("k", "abd") is None
    assert bench.traffic_from_profiles("missing", "abc") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU only" in r.stdout + r.stderr


def test_rare_target_by_hand():
    """The recycling target of the batched rare-event workload from a
    pilot ensemble: species 0 has the larger weighted mean (0.2*9 + 0.3*2 =
    2.4 against species 1's 0.2*3 + 0.5*1 + 0.3*2 = 1.7); A is the heaviest
    walker (slot 1); the threshold is the smallest t >= c_A + 2 with
    P(c >= t) <= tail."""
    import numpy as np
    x = np.array([[9, 3], [0, 1], [2, 2]])
    w = np.array([0.2, 0.5, 0.3])
    sp, xa, thr = wl.rare_target(x, w, tail=0.25)
    assert sp == 0
    assert list(xa) == [0, 1]
    # c_A = 0: t = 2 has P(c >= 2) = 0.5 > 0.25; t = 3 has 0.2 <= 0.25
    assert thr == 3
    sp, xa, thr = wl.rare_target(x, w, tail=0.1)
    assert thr == 10            # nothing is left at or above 10 (max count 9, P(c >= 10) = 0)
    cfg = wl.rare_batch_config(wl.batch_configs(n_runs=2, n_iters=10)[1], 0.5, 0, np.array([4, 1] + [0] * 6, np.int32), 12)
    assert cfg.recycle and cfg.tgt_thr == 12.0 and cfg.a_thr == 4.0
    assert cfg.edges[0] == 4.0 and cfg.edges[-1] == 12.0 and len(cfg.edges) == 17
    assert cfg.bin_coef[0] == 1.0 and cfg.bin_coef.sum() == 1.0


def test_batch_tau_scales_to_ten_events():
    assert wl.batch_tau(1.0) == 0.1
    assert wl.batch_tau(100.0) == 0.01          # clipped below
    assert wl.batch_tau(0.0) == 5.0             # clipped above
    assert abs(wl.batch_tau(2.0, tau0=0.3) - 1.5) < 1e-15


def test_weighted_logit_edges_keep_ends_order_and_symmetry():
    """Equal weight per unit logit on edges symmetric about z = 0: the new
    inner edges keep the first and last inner edge, increase strictly, stay
    symmetric, and crowd towards z = 0, where q (1 - q) is largest."""
    import numpy as np
    e = np.linspace(-9.0, 9.0, 65)
    w = np.diff(e)
    out = bench._weighted_logit_edges(e, w)
    assert out[1] == e[1] and out[-2] == e[-2] and out[0] == e[0] and out[-1] == e[-1]
    assert np.all(np.diff(out[1:-1]) > 0)
    assert np.allclose(out, -out[::-1], atol=1e-9)
    assert np.diff(out[31:34]).max() < np.diff(e[31:34]).min()
    # a bin without weight still gets a positive width
    w2 = w.copy()
    w2[10:20] = 0.0
    assert np.all(np.diff(bench._weighted_logit_edges(e, w2)[1:-1]) > 0)
