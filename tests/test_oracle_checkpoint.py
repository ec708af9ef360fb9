"""Failure and recovery on the CPU: an oracle WE run killed after an
iteration and restored from its checkpoint continues bit for bit as the
uninterrupted run.  An iteration boundary is a consistent cut (the WE
procedure saves coordinates and weights after every iteration, Sec. II.B),
and the random numbers are keyed by (seed, slot, event, iteration), so the
ensemble, the iteration and the series are the whole state."""
import dataclasses
import os
import signal
import subprocess
import sys

import numpy as np

from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import dataclasses, os, signal, sys
sys.path.insert(0, {root!r})
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl
cfg = dataclasses.replace(wl.schlogl_config(n_runs=1, seed0=9, n_iters=60), resample_rule=1)
o = orc.OracleWE(cfg, 9, rw_period=5)
o.step({k})
o.save({path!r})
os.kill(os.getpid(), signal.SIGKILL)      # the process dies right after the checkpoint
o.step(1000)                              # never reached
"""


def test_killed_oracle_resumes_bit_identically(tmp_path):
    k, total = 23, 40
    path = str(tmp_path / "ckpt.npz")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, k=k, path=path)])
    assert r.returncode == -signal.SIGKILL
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=1, seed0=9, n_iters=60), resample_rule=1)
    resumed = orc.OracleWE.load(cfg, path, rw_period=5)
    assert resumed.iter == k
    resumed.step(total - k)
    ref = orc.OracleWE(cfg, 9, rw_period=5)
    ref.step(total)
    for a, b in zip(resumed.walkers(), ref.walkers()):
        assert np.array_equal(a, b)
    assert resumed.flux == ref.flux and resumed.events == ref.events
    assert resumed.segments == ref.segments
    assert np.array_equal(resumed.rw_F, ref.rw_F)
    assert (resumed.rw_applied, resumed.rw_skipped) == (ref.rw_applied, ref.rw_skipped)
