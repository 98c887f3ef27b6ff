"""Degree-parameter optimisation (Section 2.6, Equation 2).

The loss L(e_o, e_i, p_l, p_u) is the mean of log10 C over the target
precision range, where C is the mean number of distance computations of a
search whose mean precision is p.  It is measured, as the paper does, from
actual searches: binary searches find a range eps_l whose precision lies in
(p_l - 0.005, p_l] and eps_u whose precision lies in [p_u, p_u + 0.005);
ten ranges spaced evenly over [eps_l, eps_u] give ten (p, C) samples, and the
trapezoidal rule over them gives the integral.  The integral runs over the
samples' own precision span and is divided by that span (the printed formula
divides by p_u - p_l; the samples cover the target range up to the 0.005
brackets).  L is minimised over (e_o, e_i) by hill climbing in steps of 5
(Section 3.2), which the paper justifies by L being convex (Figure 3b).

Host orchestration only: every search and graph build it drives runs in the
library's kernels, through caller-supplied functions, and the loss of the
samples is the library's onng_degree_loss.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Optional, Tuple

BRACKET = 0.005


def _find_range(search: Callable[[float], Tuple[float, float]], target: float, upper: bool,
                lo: float, hi: float, iters: int) -> Optional[float]:
    """Binary search for a range whose precision p lands in the bracket:
    [target, target + 0.005) for the upper end, (target - 0.005, target] for
    the lower.  Precision is taken to grow with the range."""
    p_lo = search(lo)[0]
    if not upper and p_lo > target:
        return lo                    # already above the lower target at the smallest range
    p_hi = search(hi)[0]
    if p_hi < target:
        return None                  # the target is out of reach
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        p = search(mid)[0]
        if upper:
            if p < target:
                lo = mid
            elif p >= target + BRACKET:
                hi = mid
            else:
                return mid
        else:
            if p > target:
                hi = mid
            elif p <= target - BRACKET:
                lo = mid
            else:
                return mid
    return hi if upper else lo


def degree_loss(search: Callable[[float], Tuple[float, float]], p_l: float = 0.90,
                p_u: float = 0.98, eps_max: float = 1.0, iters: int = 30,
                samples: int = 10) -> Tuple[float, list]:
    """L of one graph.  search(eps) returns (mean precision, mean distance
    computations) of the queries at range eps.  Returns (L, samples as
    (eps, p, C)); L is +inf when p_u is not reached."""
    eu = _find_range(search, p_u, True, 0.0, eps_max, iters)
    if eu is None:
        return math.inf, []
    el = _find_range(search, p_l, False, 0.0, eu, iters)
    pts = []
    for i in range(samples):
        e = el + (eu - el) * i / (samples - 1)
        p, c = search(e)
        pts.append((e, p, c))
    from . import api
    return api.degree_loss_from_samples([p for _, p, _ in pts], [c for _, _, c in pts]), pts


def hill_climb(loss: Callable[[int, int], float], e_o: int, e_i: int, step: int = 5,
               max_moves: int = 50) -> Tuple[Tuple[int, int], float, Dict[Tuple[int, int], float]]:
    """Move to the best of the four neighbours (e_o +- step, e_i +- step) while
    it lowers the loss.  Returns the final point, its loss and every
    evaluation."""
    seen: Dict[Tuple[int, int], float] = {}

    def ev(pt):
        if pt not in seen:
            seen[pt] = loss(*pt)
        return seen[pt]

    cur = (e_o, e_i)
    best = ev(cur)
    for _ in range(max_moves):
        nbrs = [(cur[0] + a, cur[1] + b) for a, b in ((step, 0), (-step, 0), (0, step), (0, -step))
                if cur[0] + a >= 1 and cur[1] + b >= 0]
        cand = min(nbrs, key=ev)
        if ev(cand) < best:
            cur, best = cand, ev(cand)
        else:
            break
    return cur, best, seen
