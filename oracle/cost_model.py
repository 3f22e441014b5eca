"""The paper's analytic cost formulas, in float64 -- TEST INFRASTRUCTURE ONLY.

Each function restates one formula of the paper; costs count tuples read
onto the accelerator chip.  ``M`` is the on-chip capacity in tuples, the
bucket-count names (H, G, g, h, d) follow the paper's notation (Sec. 3.1):
a hash function's name also stands for its number of buckets.

Readings where the text is ambiguous:
  * Example 4 prints the cyclic inequality without the factor 2 that the
    derivation of Sec. 5.2 gives; both are provided
    (``cyclic_example_threshold_printed`` / ``cyclic_threshold``).
  * The number of comparisons of the cascade's second join is taken as
    |I||T|/g (the loop-nest count of App. A and the star footnote of
    Sec. 6.5), the expected number of matches as |I||T|/d.
"""
from __future__ import annotations

import math


def linear_tuples_read(R: float, S: float, T: float, M: float) -> float:
    """Linear 3-way join, Sec. 4.2: R and S are read once, T once per
    partition of R, and R has |R|/M partitions: |R| + |S| + |R||T|/M."""
    return R + S + R * T / M


def cascade_tuples_moved(I: float) -> float:
    """Cascade of two binary joins (Example 3): the intermediate is written
    out and read back in, 2|I| tuples."""
    return 2.0 * I


def linear_threshold(R: float, S: float, T: float, I: float) -> float:
    """Smallest M for which the 3-way join reads fewer tuples than the
    cascade moves (Example 3): |R|+|S|+|R||T|/M < 2|I|  <=>
    M > |R||T| / (2|I| - |R| - |S|).  Returns +inf when no M suffices."""
    room = 2.0 * I - R - S
    return math.inf if room <= 0 else R * T / room


def cyclic_tuples_read(R: float, S: float, T: float, M: float, H: float) -> float:
    """Cyclic 3-way join, Sec. 5.2: |R| + H|S| + G|T| with GH = |R|/M,
    i.e. |R| + H|S| + |R||T|/(M H)."""
    G = R / (M * H)
    return R + H * S + G * T


def cyclic_optimal_H(R: float, S: float, T: float, M: float) -> float:
    """Minimiser of the cyclic cost over H (Sec. 5.2): sqrt(|R||T| / (M|S|))."""
    return math.sqrt(R * T / (M * S))


def cyclic_min_tuples_read(R: float, S: float, T: float, M: float) -> float:
    """Cyclic cost at the optimal H (Sec. 5.2): |R| + 2 sqrt(|R||S||T|/M)."""
    return R + 2.0 * math.sqrt(R * S * T / M)


def cyclic_threshold(R: float, S: float, T: float, budget: float) -> float:
    """Smallest M with |R| + 2 sqrt(|R||S||T|/M) < budget (the derived form)."""
    room = (budget - R) / 2.0
    return math.inf if room <= 0 else R * S * T / (room * room)


def cyclic_example_threshold_printed(F: float, budget: float) -> float:
    """Example 4 as printed: F(1 + sqrt(F/M)) < budget  <=>  M > F / (budget/F - 1)^2."""
    q = budget / F - 1.0
    return math.inf if q <= 0 else F / (q * q)


def join2_size_uniform(R: float, S: float, d: float) -> float:
    """Estimated size of R join S under uniform keys with d distinct values
    (Sec. 6.3): |R||S|/d."""
    return R * S / d


def cascade_join2_loaded(I: float, T: float) -> float:
    """Tuples loaded by the cascade's second join (Sec. 6.3): |R join S| + |T|."""
    return I + T


def cascade_join2_comparisons(I: float, T: float, g: float) -> float:
    """Comparisons of the second join with g buckets on C: |I||T|/g."""
    return I * T / g


def cascade_join2_matches(I: float, T: float, d: float) -> float:
    """Expected matches of the second join: |I||T|/d."""
    return I * T / d


def star_cascade_comparisons(R: float, S: float, T: float, d: float,
                             h: float, g: float) -> float:
    """Comparisons of the cascade for the star join (Sec. 6.5 footnote):
    |R||S|/h + |R||S||T|/(d g)."""
    return R * S / h + R * S * T / (d * g)


def branch_hit_probability(g3: float, d: float) -> float:
    """App. A: S-T comparisons number |S||T|/g3 while |S||T|/d of them match,
    so the branch on S.C == T.C is taken with probability g3/d."""
    return g3 / d


def comparisons_3way_ST(S: float, T: float, H3: float, h3: float, g3: float) -> float:
    """App. A: loop trip product enclosing the S.C == T.C branch,
    H3 h3 g3 (|T|/g3) (|S|/(H3 g3 h3)) = |S||T|/g3."""
    return H3 * h3 * g3 * (T / g3) * (S / (H3 * g3 * h3))
