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
    """Philox 100 + uniforms 10 + waiting time 5 + target/time 2, and per
    reaction 5 + f_j: A+2X->3X (C(x,2): 3), 3X->A+2X (C(x,3): 6), B->X (0),
    X->B (0), so 4 x 5 + 9 = 29; one changed species + 2 bound checks."""
    assert bench.alg_ops_per_event(wl.schlogl()) == 100 + 10 + 5 + 2 + 29 + 1 + 2 == 149


def test_ops_per_event_two_species_reaction():
    """A + B -> C adds the two-species product (1) to 5; mean changed
    species 3."""
    net = wl.Network.from_reactions(["A", "B", "C"], [({"A": 1, "B": 1}, {"C": 1}, 1.0)])
    assert bench.alg_ops_per_event(net) == 100 + 10 + 5 + 2 + 6 + 3 + 2


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
