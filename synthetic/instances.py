"""Seeded problem instances: graphs, couplings and the annealing schedule.

The paper's workloads are random 3-regular graphs with random couplings
(Sec. III.B).  Here the graph comes from the configuration model with
rejection and the couplings are uniform on a dyadic grid, all drawn from one
SplitMix64 stream so that any language can regenerate the same instance.

Conventions (shared by every consumer of an instance):

* SplitMix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15, then the
  usual two xor-shift-multiply rounds and a final xor-shift.
* Bounded integers in [0, m): draw, keep the low bits under the smallest
  all-ones mask that covers m-1, reject and redraw when the value is >= m.
* Configuration model: stubs 0..3n-1 in order (stub s belongs to vertex s//3),
  Fisher-Yates from the top (for i = 3n-1 .. 1 swap i with bounded(i+1)),
  pair stubs (2t, 2t+1).  A pairing with a self-loop or a repeated edge is
  thrown away and the draw repeats on the same stream.
* Edges are stored with u < v and sorted lexicographically; an edge's id is
  its rank in that order.
* After the graph, J[e] for e = 0..|E|-1 and then h[a] for a = 0..n-1, each
  ((x >> 39) - 2**24) * 2**-24, i.e. uniform on the 2**-24 grid of [-1, 1).
  Every coupling is a multiple of 2**-24 with magnitude <= 1, so any sum of
  them up to a few thousand terms is exact in binary64.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """64-bit SplitMix generator (Steele, Lea, Flood, OOPSLA 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def bounded(self, m: int) -> int:
        """Uniform integer in [0, m) by bit-mask rejection."""
        if m <= 0:
            raise ValueError("bound must be positive")
        if m == 1:
            return 0
        mask = (1 << (m - 1).bit_length()) - 1
        while True:
            x = self.next() & mask
            if x < m:
                return x

    def grid_unit(self) -> float:
        """Uniform value on the 2**-24 grid of [-1, 1)."""
        return grid_coupling(self.next())


def grid_coupling(x: int) -> float:
    return float((x >> 39) - (1 << 24)) * 2.0 ** -24


def splitmix64_at(seed: int, i: int) -> int:
    """Output i (0-based) of SplitMix64(seed), by counter: the state after
    i + 1 steps is seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2**64)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def random_message_entries(seed: int, dims, chi: int):
    """Random d x d complex matrices A, one per edge direction, for a random
    BP start (entries[e][dir], d = dims[e]).  Entry A[r][k] of direction dir
    of edge e takes outputs 2i and 2i + 1 of SplitMix64(seed) as real and
    imaginary parts, i = ((e * 2 + dir) * chi + r) * chi + k, each mapped to
    (x >> 11) * 2**-52 - 1, uniform on the 2**-52 grid of [-1, 1)."""
    def u(x):
        return float(x >> 11) * 2.0 ** -52 - 1.0
    out = []
    for e, d in enumerate(dims):
        pair = []
        for dr in range(2):
            A = np.zeros((d, d), dtype=np.complex128)
            for r in range(d):
                for k in range(d):
                    i = 2 * (((e * 2 + dr) * chi + r) * chi + k)
                    A[r, k] = complex(u(splitmix64_at(seed, i)), u(splitmix64_at(seed, i + 1)))
            pair.append(A)
        out.append(pair)
    return out


@dataclass
class Instance:
    """An Ising problem on a graph: E(x) = sum_e J_e x_u x_v + sum_a h_a x_a."""

    n: int
    edges: np.ndarray          # int32 [E, 2], u < v, lexicographically sorted
    J: np.ndarray              # float64 [E]
    h: np.ndarray              # float64 [n]
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def degrees(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.int64)
        np.add.at(d, self.edges[:, 0], 1)
        np.add.at(d, self.edges[:, 1], 1)
        return d


def _sorted_edges(pairs) -> np.ndarray:
    norm = sorted((min(u, v), max(u, v)) for u, v in pairs)
    return np.asarray(norm, dtype=np.int32).reshape(-1, 2)


def random_regular_instance(seed: int, n: int, degree: int = 3,
                            couplings: str = "grid") -> Instance:
    """Uniform simple d-regular graph by the configuration model with rejection."""
    if n <= degree or (n * degree) % 2:
        raise ValueError("need n > degree and n*degree even")
    rng = SplitMix64(seed)
    n_stubs = n * degree
    attempts = 0
    while True:
        attempts += 1
        stubs = list(range(n_stubs))
        for i in range(n_stubs - 1, 0, -1):
            j = rng.bounded(i + 1)
            stubs[i], stubs[j] = stubs[j], stubs[i]
        seen = set()
        ok = True
        for t in range(n_stubs // 2):
            u = stubs[2 * t] // degree
            v = stubs[2 * t + 1] // degree
            if u == v:
                ok = False
                break
            key = (min(u, v), max(u, v))
            if key in seen:
                ok = False
                break
            seen.add(key)
        if ok:
            break
    edges = _sorted_edges(seen)
    J, h = _draw_couplings(rng, edges.shape[0], n, couplings)
    return Instance(n=n, edges=edges, J=J, h=h, seed=seed,
                    meta={"kind": f"random-{degree}-regular", "attempts": attempts})


def random_tree_instance(seed: int, n: int, max_degree: int = 3,
                         couplings: str = "grid") -> Instance:
    """Random tree with degrees <= max_degree: vertex a >= 1 attaches to a
    uniformly chosen earlier vertex that still has a free slot."""
    rng = SplitMix64(seed)
    deg = [0] * n
    pairs = []
    for a in range(1, n):
        cands = [b for b in range(a) if deg[b] < max_degree]
        b = cands[rng.bounded(len(cands))]
        pairs.append((b, a))
        deg[a] += 1
        deg[b] += 1
    edges = _sorted_edges(pairs)
    J, h = _draw_couplings(rng, edges.shape[0], n, couplings)
    return Instance(n=n, edges=edges, J=J, h=h, seed=seed, meta={"kind": "tree"})


def instance_from_edges(n: int, pairs, seed: int = 0, couplings: str = "grid",
                        J=None, h=None) -> Instance:
    """Instance on a given edge list; couplings drawn from `seed` unless given."""
    edges = _sorted_edges(pairs)
    rng = SplitMix64(seed)
    Jd, hd = _draw_couplings(rng, edges.shape[0], n, couplings)
    if J is not None:
        Jd = np.asarray(J, dtype=np.float64).copy()
    if h is not None:
        hd = np.asarray(h, dtype=np.float64).copy()
    return Instance(n=n, edges=edges, J=Jd, h=hd, seed=seed, meta={"kind": "given"})


def _draw_couplings(rng: SplitMix64, n_edges: int, n: int, couplings: str):
    if couplings == "grid":
        J = np.array([rng.grid_unit() for _ in range(n_edges)], dtype=np.float64)
        h = np.array([rng.grid_unit() for _ in range(n)], dtype=np.float64)
    elif couplings == "maxcut":
        J = -np.ones(n_edges, dtype=np.float64)
        h = np.zeros(n, dtype=np.float64)
    elif couplings == "zero-j":
        J = np.zeros(n_edges, dtype=np.float64)
        h = np.array([rng.grid_unit() for _ in range(n)], dtype=np.float64)
    else:
        raise ValueError(couplings)
    return J, h


def schedule_angles_second_order(T: float, dt: float):
    """Angles of the symmetric (second-order) product formula for the same
    linear schedule, sampled at step midpoints s_k = (k - 1/2)/K: interaction
    angle dt*s_k and mixing half-angles a_k = dt*(1 - s_k)/2.  Returns
    (theta_z[K], theta_x[K], theta_x0): a lone mixing layer theta_x0 = a_1,
    then K steps (interaction theta_z[k], mixing theta_x[k] = a_k + a_(k+1),
    a_(K+1) = 0), i.e. the product of X(a_k) Z(dt*s_k) X(a_k) over k with
    adjacent half-layers merged."""
    K = int(round(T / dt))
    s = np.array([(k - 0.5) / K for k in range(1, K + 1)], dtype=np.float64)
    tz = dt * s
    a = 0.5 * dt * (1.0 - s)
    tx = a + np.concatenate([a[1:], [0.0]])
    return tz, tx, float(a[0])


def schedule_angles_randomised(T: float, dt: float, x_first):
    """Angles of the randomised first-order product formula for the same
    linear schedule: step k applies Z(dt*s_k) and X(dt*(1 - s_k)) at the
    midpoint s_k = (k - 1/2)/K, mixing layer first iff x_first[k] (the random
    choices, drawn by the caller: fair coins give an averaged channel of
    second order).  Returned in the form (theta_z[K], theta_x[K], theta_x0)
    of a lone mixing layer followed by K interaction-then-mixing steps:
    a mixing layer applied first joins the previous step's mixing angle (or
    theta_x0 at k = 1)."""
    K = int(round(T / dt))
    xf = np.asarray(x_first, dtype=bool).ravel()
    if xf.size != K:
        raise ValueError(f"x_first needs one choice per step ({K})")
    s = np.array([(k - 0.5) / K for k in range(1, K + 1)], dtype=np.float64)
    tz = dt * s
    ax = dt * (1.0 - s)
    tx = np.zeros(K, dtype=np.float64)
    tx0 = 0.0
    for k in range(K):
        if not xf[k]:
            tx[k] += ax[k]
        elif k == 0:
            tx0 += ax[k]
        else:
            tx[k - 1] += ax[k]
    return tz, tx, float(tx0)


def schedule_angles(T: float, dt: float):
    """Per-step (theta_z, theta_x) of the linear schedule s(t) = 1 - t/T sampled
    at the right end of each step: K = round(T/dt), theta_z = dt*k/K,
    theta_x = dt*(K-k)/K for k = 1..K (App. F, first-order product formula)."""
    K = int(round(T / dt))
    tz = np.array([dt * k / K for k in range(1, K + 1)], dtype=np.float64)
    tx = np.array([dt * (K - k) / K for k in range(1, K + 1)], dtype=np.float64)
    return tz, tx
