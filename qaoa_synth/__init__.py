"""Seeded synthetic QAOA MaxCut instances: random d-regular graphs and angles.

This module is the only code shared by the FP64 oracle and the HIP path.  It
draws random numbers and builds edge lists; it holds none of the method's
arithmetic (no gates, no tensors, no contraction).

Random numbers come from xoshiro256** seeded through splitmix64 (Blackman and
Vigna, "Scrambled linear pseudorandom number generators", 2018), written here
from their published definitions.  Bounded integers use Lemire's
multiply-and-reject method (Lemire, "Fast random integer generation in an
interval", 2019).

Graphs follow the pairing (configuration) model: N*d half-edge points are
matched by a uniform shuffle and the whole sample is rejected if it has a
self-loop or a repeated edge, so an accepted graph is uniform over simple
d-regular graphs.  The paper's benchmark graphs are random 3-regular graphs
(Sec. II-E); QAOA angles gamma_k ~ U[0, pi), beta_k ~ U[0, pi/2) are drawn
after the graph from the same stream, all gammas first, then all betas.
"""

from __future__ import annotations

import math

MASK64 = (1 << 64) - 1


def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & MASK64


class SplitMix64:
    """splitmix64: a 64-bit Weyl sequence followed by a variant of the
    MurmurHash3 finaliser (used only to expand a seed into xoshiro state)."""

    def __init__(self, seed: int):
        self.x = seed & MASK64

    def next(self) -> int:
        self.x = (self.x + 0x9E3779B97F4A7C15) & MASK64
        z = self.x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


class Rng:
    """xoshiro256** generator."""

    def __init__(self, seed: int):
        sm = SplitMix64(seed)
        self.s = [sm.next() for _ in range(4)]

    def next_u64(self) -> int:
        s = self.s
        result = (_rotl((s[1] * 5) & MASK64, 7) * 9) & MASK64
        t = (s[1] << 17) & MASK64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
        return result

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def below(self, n: int) -> int:
        """Unbiased integer in [0, n), n >= 1."""
        if n <= 0:
            raise ValueError("below() needs n >= 1")
        m = self.next_u64() * n
        low = m & MASK64
        if low < n:
            threshold = ((1 << 64) - n) % n
            while low < threshold:
                m = self.next_u64() * n
                low = m & MASK64
        return m >> 64


def random_regular_graph(rng: Rng, n: int, d: int, max_tries: int = 100000):
    """Uniform simple d-regular graph on n vertices by the pairing model.

    Returns the edge list as sorted (u, v) pairs with u < v.
    """
    if n <= d or (n * d) % 2 != 0:
        raise ValueError(f"no simple {d}-regular graph on {n} vertices")
    pts = n * d
    for _ in range(max_tries):
        perm = list(range(pts))
        for i in range(pts - 1, 0, -1):
            j = rng.below(i + 1)
            perm[i], perm[j] = perm[j], perm[i]
        seen = set()
        ok = True
        for i in range(0, pts, 2):
            a, b = perm[i] // d, perm[i + 1] // d
            if a == b:
                ok = False
                break
            e = (a, b) if a < b else (b, a)
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted(seen)
    raise RuntimeError("pairing model did not produce a simple graph")


def qaoa_angles(rng: Rng, p: int):
    """gamma_k ~ U[0, pi), beta_k ~ U[0, pi/2), k = 1..p."""
    gamma = [math.pi * rng.uniform() for _ in range(p)]
    beta = [0.5 * math.pi * rng.uniform() for _ in range(p)]
    return gamma, beta


def instance(n: int, d: int, p: int, seed: int, n_angle_sets: int = 1):
    """One graph and ``n_angle_sets`` angle sets from one seeded stream."""
    rng = Rng(seed)
    edges = random_regular_graph(rng, n, d)
    angles = [qaoa_angles(rng, p) for _ in range(n_angle_sets)]
    return {"n": n, "d": d, "p": p, "seed": seed, "edges": edges,
            "angles": angles}


def batch_instances(master_seed: int, count: int, n_lo: int, n_hi: int,
                    p_choices, d: int = 3):
    """``count`` graphs with N uniform over the admissible sizes in
    [n_lo, n_hi] (even N when d is odd) and p uniform over ``p_choices``.
    Each graph gets its own sub-seed drawn from the master stream."""
    master = Rng(master_seed)
    sizes = [n for n in range(n_lo, n_hi + 1) if (n * d) % 2 == 0 and n > d]
    out = []
    for _ in range(count):
        n = sizes[master.below(len(sizes))]
        p = list(p_choices)[master.below(len(p_choices))]
        sub = master.next_u64()
        out.append(instance(n, d, p, sub, 1))
    return out


def petersen_graph():
    """The Petersen graph: 3-regular, 10 vertices, 15 edges, girth 5
    (triangle-free).  Outer 5-cycle 0..4, spokes i--i+5, inner pentagram."""
    e = []
    for i in range(5):
        e.append((i, (i + 1) % 5))
        e.append((i, i + 5))
        e.append((5 + i, 5 + (i + 2) % 5))
    return sorted((min(a, b), max(a, b)) for a, b in e)


def edges_flat(edges):
    """Edge list as a flat [u0, v0, u1, v1, ...] list of ints."""
    out = []
    for a, b in edges:
        out.extend((int(a), int(b)))
    return out
