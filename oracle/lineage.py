"""Committor labels from WE lineages, written as a plain loop (test
infrastructure only).

Given the resampled ensembles of consecutive iterations -- per iteration and
run: states x[k], parent slots origin[k] (slots of the previous iteration)
and whether the parent reached B in that interval -- every walker's counts
(n_A, n_B) are the first outcomes of its children: B if the child's parent
was recycled, A if the child lies in A = {x : a_coef . x <= a_thr},
otherwise the child's own counts.  Walkers of the last iteration have none.
"""
import numpy as np


def label_counts(records, a_coef, a_thr):
    """records: list over iterations of (n[run], x[run][slot][S],
    origin[run][slot], recycled[run][slot]).  Returns counts shaped
    [iters][runs][slots][2] (uint32)."""
    a_coef = np.asarray(a_coef, np.float64)
    T = len(records)
    n0, x0, _, _ = records[0]
    runs, cap, S = x0.shape
    cnt = np.zeros((T, runs, cap, 2), np.uint32)
    for i in range(T - 1, 0, -1):
        n, x, origin, rec = records[i]
        for r in range(runs):
            for k in range(int(n[r])):
                if rec[r, k]:
                    add = (0, 1)
                else:
                    q = 0.0
                    for s in range(S):
                        q = q + a_coef[s] * float(x[r, k, s])
                    add = (1, 0) if q <= a_thr else (int(cnt[i, r, k, 0]), int(cnt[i, r, k, 1]))
                p = int(origin[r, k])
                cnt[i - 1, r, p, 0] += add[0]
                cnt[i - 1, r, p, 1] += add[1]
    return cnt
