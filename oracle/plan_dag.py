"""Reference model of the paper's mixed-radix schedule search -- TEST INFRASTRUCTURE ONLY.

Paper, Approach, bottom-level analysis ("FFT performance model"):

* A schedule of an FFT of 2^L points is a sequence of radices r_1..r_m
  (each a power of two up to the largest radix) with sum(log2 r_i) = L.
* The states are the stage indices 0..L; a radix-r stage starting at stage s
  is an edge s -> s + log2(r).  Every source-to-sink path is a valid schedule,
  so the number of schedules is the number of paths.
* Hypothesis: a stage's cost depends only on its radix and its start stage,
  so a schedule's cost is the sum of its edge costs and the best schedule is
  the shortest path (the paper uses Dijkstra's algorithm).
* The benchmark set is one run per (radix, start stage): for radices 2, 4, 8
  that is L + (L-1) + (L-2) = 3(L-1) runs.

This module writes those statements out with plain Python so the product's
C++ autotuner can be checked against it.
"""
from __future__ import annotations

import heapq
import math
from typing import Dict, List, Optional, Sequence, Tuple

Costs = Dict[Tuple[int, int], float]   # (radix, start_stage) -> cost


def count_schedules(log2n: int, radices: Sequence[int] = (2, 4, 8)) -> int:
    """Number of source-to-sink paths of the stage DAG (counted by brute-force enumeration)."""
    steps = [int(math.log2(r)) for r in radices]
    return sum(1 for _ in enumerate_schedules(log2n, radices)) if log2n <= 16 else \
        _count_dp(log2n, steps)


def _count_dp(log2n: int, steps: Sequence[int]) -> int:
    ways = [0] * (log2n + 1)
    ways[0] = 1
    for s in range(1, log2n + 1):
        ways[s] = sum(ways[s - d] for d in steps if s - d >= 0)
    return ways[log2n]


def enumerate_schedules(log2n: int, radices: Sequence[int] = (2, 4, 8)):
    """Yield every radix list whose log2 sizes sum to log2n (depth-first, in radix order)."""
    def rec(at: int, acc: List[int]):
        if at == log2n:
            yield list(acc)
            return
        for r in radices:
            d = int(math.log2(r))
            if at + d <= log2n:
                acc.append(r)
                yield from rec(at + d, acc)
                acc.pop()
    yield from rec(0, [])


def stage_runs(log2n: int, radices: Sequence[int] = (2, 4, 8)) -> int:
    """Benchmarks needed: one per (radix, start stage) that fits before the sink."""
    return sum(log2n - int(math.log2(r)) + 1 for r in radices if int(math.log2(r)) <= log2n)


def schedule_cost(schedule: Sequence[int], costs: Costs) -> float:
    """Additive cost of a schedule: the sum of its (radix, start stage) entries."""
    at, total = 0, 0.0
    for r in schedule:
        total += costs[(r, at)]
        at += int(math.log2(r))
    return total


def dijkstra(log2n: int, costs: Costs, radices: Optional[Sequence[int]] = None):
    """Shortest source-to-sink path over the stage DAG with Dijkstra's algorithm.

    Returns (cost, schedule).  Ties between equal-cost paths go to the one
    with fewer stages, then to the lexicographically larger radix list.
    """
    if radices is None:
        radices = sorted({r for (r, _) in costs})
    # key: (cost, n_stages, negated radix list) -> smallest is best
    best: Dict[int, Tuple[float, int, Tuple[int, ...]]] = {0: (0.0, 0, ())}
    heap = [(0.0, 0, (), 0)]
    done = set()
    while heap:
        c, nst, negs, node = heapq.heappop(heap)
        if node in done:
            continue
        done.add(node)
        if node == log2n:
            return c, [-v for v in negs]
        for r in radices:
            d = int(math.log2(r))
            if node + d > log2n or (r, node) not in costs:
                continue
            cand = (c + costs[(r, node)], nst + 1, negs + (-r,))
            nxt = node + d
            if nxt not in best or cand < best[nxt]:
                best[nxt] = cand
                heapq.heappush(heap, (cand[0], cand[1], cand[2], nxt))
    raise ValueError("no schedule reaches the sink")


def brute_force_best(log2n: int, costs: Costs, radices: Sequence[int] = (2, 4, 8)):
    """Minimum over every enumerated schedule (same tie rule as ``dijkstra``)."""
    best = None
    for s in enumerate_schedules(log2n, radices):
        try:
            c = schedule_cost(s, costs)
        except KeyError:
            continue
        key = (c, len(s), tuple(-r for r in s))
        if best is None or key < best[0]:
            best = (key, s)
    return best[0][0], best[1]


def load_stage_table(path: str) -> Costs:
    """Parse a ``stage radix2 radix4 radix8`` table; X entries are skipped."""
    costs: Costs = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            stage = int(parts[0])
            for r, tok in zip((2, 4, 8), parts[1:]):
                if tok != "X":
                    costs[(r, stage)] = float(tok)
    return costs
