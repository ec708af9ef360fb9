"""Analysis formulas of the paper, written plainly (test infrastructure only).

censored_mle: Eq. mld (Sec. II.C).  The printed first line,
(1 - n/N) T + (1/n) sum t_i, does not reproduce the paper's own numbers
(Sec. III.C: N = 753 runs of T = 1e6 s give mu = 1.3e6 s, sigma = 6.5e4 s).
The maximum-likelihood estimate of an exponential mean from n observed
passage times and N - n runs censored at T is
    mu = ((N - n) T + sum t_i) / n = ((N - n)/n) T + (1/n) sum t_i,
with standard error mu / sqrt(n); this reading reproduces both printed values.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple


def censored_mle(T: float, N: int, times: Sequence[float]) -> Tuple[float, float]:
    n = len(times)
    if n == 0:
        return float("inf"), float("inf")
    mu = ((N - n) / n) * T + sum(times) / n
    return mu, mu / math.sqrt(n)


def censored_mle_as_printed(T: float, N: int, times: Sequence[float]) -> float:
    """Eq. mld exactly as typeset (kept only to document the reading)."""
    n = len(times)
    return (1.0 - n / N) * T + sum(times) / n
