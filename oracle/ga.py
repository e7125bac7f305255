"""Oracle of the genetic search -- TEST INFRASTRUCTURE (tests only).

The paper's search (sections 3.2 and 4; parameters in section 5.1.2), written
step by step in the paper's order, with plain Python integers and lists:

1. Each gene is L bits. The initial population has M genes with every bit
   drawn 0 or 1 at random.
2. Each generation:
   a. every individual is measured and gets fitness (time)^(-1/2). A failed
      measurement, or one beyond the time limit, counts as 1000 s.
      Identical genes are measured once.
   b. the individual with the highest fitness is copied unchanged into the
      next generation (elitism).
   c. the rest of the next generation is bred. Two parents are chosen by
      roulette on fitness. They are crossed over with probability Pc, and
      every bit of each child is flipped with probability Pm.
3. After T generations the best individual measured is the answer.

Where the paper leaves a detail open, this oracle reads it as follows:
- crossover is one-point, at a point drawn uniformly from 1..L-1, with the
  low bits taken from the first parent;
- a pair of parents gives two children, and the second is dropped when the
  generation is full;
- ties go to the lowest index, or to the first measured.

Random numbers: number n of stream s under seed q is the n-th output of the
SplitMix64 generator (Steele, Lea and Flood 2014), started at state
mix(q + (s+1)*GAMMA) and reduced to [0,1) by its top 53 bits. The streams:
- stream 0 holds the initial bits (individual m, bit b at n = m*L + b);
- the step from generation g to g+1 uses stream 1+4g for roulette draws,
  2+4g for the crossover decision of each pair, 3+4g for its crossover
  point, and 4+4g for mutation (child c, bit b at n = c*L + b).
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Sequence, Tuple

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
FAIL_TIME = 1000.0


def splitmix_finalize(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix_output(state: int, n: int) -> int:
    """The n-th (0-based) output of SplitMix64 started at `state`."""
    return splitmix_finalize((state + (n + 1) * GAMMA) & MASK64)


def uniform(seed: int, stream: int, n: int) -> float:
    state = splitmix_finalize((seed + (stream + 1) * GAMMA) & MASK64)
    return (splitmix_output(state, n) >> 11) * 2.0 ** -53


def fitness(time_s: float) -> float:
    """The paper's fitness: (processing time)^(-1/2)."""
    return 1.0 / math.sqrt(time_s)


def roulette(fit: Sequence[float], total: float, u: float) -> int:
    """Index picked by a roulette wheel whose slots are sized by fitness."""
    target = u * total
    acc = 0.0
    for m, f in enumerate(fit):
        acc += f
        if target < acc:
            return m
    return len(fit) - 1


def run(L: int, M: int, T: int, seed: int, pc: float, pm: float,
        time_of: Callable[[int], float]) -> Tuple[int, float, int, List[List[int]]]:
    """Returns (best gene, best time, distinct genes measured, history)."""
    # 1. initial population
    pop = []
    for m in range(M):
        g = 0
        for b in range(L):
            if uniform(seed, 0, m * L + b) < 0.5:
                g |= 1 << b
        pop.append(g)

    measured: Dict[int, float] = {}
    best_gene, best_time = None, None
    history = []
    for gen in range(T):
        history.append(list(pop))
        # 2a. measure, fitness = time^-1/2 (failures count as 1000 s)
        times = []
        for g in pop:
            if g not in measured:
                t = time_of(g)
                if not (t > 0.0) or not math.isfinite(t) or t > FAIL_TIME:
                    t = FAIL_TIME
                measured[g] = t
            times.append(measured[g])
            if best_time is None or measured[g] < best_time:
                best_gene, best_time = g, measured[g]
        fit = [fitness(t) for t in times]
        if gen == T - 1:
            break
        # 2b. elitism
        elite = max(range(M), key=lambda m: (fit[m], -m))
        nxt = [pop[elite]]
        # 2c. roulette selection, crossover, mutation
        total = 0.0
        for f in fit:
            total += f
        s_pick, s_cross, s_point, s_mut = 1 + 4 * gen, 2 + 4 * gen, 3 + 4 * gen, 4 + 4 * gen
        draw = pair = child = 0
        while len(nxt) < M:
            a = pop[roulette(fit, total, uniform(seed, s_pick, draw))]
            b = pop[roulette(fit, total, uniform(seed, s_pick, draw + 1))]
            draw += 2
            c1, c2 = a, b
            if L > 1 and uniform(seed, s_cross, pair) < pc:
                point = 1 + int(math.floor(uniform(seed, s_point, pair) * (L - 1)))
                low = (1 << point) - 1
                c1 = (a & low) | (b & ~low & ((1 << L) - 1))
                c2 = (b & low) | (a & ~low & ((1 << L) - 1))
            pair += 1
            for c in (c1, c2):
                if len(nxt) >= M:
                    break
                for bit in range(L):
                    if uniform(seed, s_mut, child * L + bit) < pm:
                        c ^= 1 << bit
                child += 1
                nxt.append(c)
        pop = nxt
    return best_gene, best_time, len(measured), history
