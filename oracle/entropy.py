"""Mean-field entanglement entropy over a balanced bipartition (Sec. III.C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* `spectral_bipartition`: the heuristic for Eq. `bipartition`
  (argmin over A of |dA| / (|A| |A-bar|)) by spectral graph partitioning:
  order the vertices by the Fiedler vector of the graph Laplacian L = D - Adj
  (the relaxation of that ratio cut) and take the best prefix of the order
  under the same ratio.  Reading: the paper names the method (spectral
  partitioning) but not the rounding of the eigenvector; the sweep over
  prefixes optimises the paper's objective directly.  Ties in the Fiedler
  values are ordered by vertex id and ties in the ratio go to the shortest
  prefix.
* `mean_field_entropy`: Eq. `apprx_entropy` with the Schmidt values of
  Eq. `mean_field_schmidt` taken from the Vidal-gauge lambdas: the sum over
  cut edges of -sum_j lambda_j^2 log lambda_j^2 (natural logarithm; lambda
  has unit 2-norm, zero entries contribute nothing).
"""

from __future__ import annotations

import numpy as np


def laplacian(n: int, edges) -> np.ndarray:
    L = np.zeros((n, n))
    for u, v in np.asarray(edges, dtype=np.int64):
        L[u, u] += 1.0
        L[v, v] += 1.0
        L[u, v] -= 1.0
        L[v, u] -= 1.0
    return L


def cut_ratio(n: int, edges, side) -> float:
    """|dA| / (|A| |A-bar|) of Eq. bipartition for side[a] in {0, 1} (A = side 1)."""
    side = np.asarray(side)
    k = int(side.sum())
    if k == 0 or k == n:
        return np.inf
    cut = sum(1 for u, v in np.asarray(edges) if side[u] != side[v])
    return cut / (k * (n - k))


def spectral_bipartition(n: int, edges):
    """side[a] = 1 for a in A*, with A* the best prefix of the Fiedler order."""
    L = laplacian(n, edges)
    w, V = np.linalg.eigh(L)
    f = V[:, 1]
    # fix the eigenvector's sign: largest |entry| positive (first such vertex)
    i = int(np.argmax(np.abs(f)))
    if f[i] < 0:
        f = -f
    order = sorted(range(n), key=lambda a: (f[a], a))
    edges = np.asarray(edges, dtype=np.int64)
    nbr = [[] for _ in range(n)]
    for u, v in edges:
        nbr[u].append(v)
        nbr[v].append(u)
    inA = np.zeros(n, dtype=bool)
    cut = 0
    best = (np.inf, 0)
    for k in range(1, n):
        a = order[k - 1]
        for b in nbr[a]:
            cut += -1 if inA[b] else 1
        inA[a] = True
        r = cut / (k * (n - k))
        if r < best[0]:
            best = (r, k)
    side = np.zeros(n, dtype=np.uint8)
    side[order[:best[1]]] = 1
    return side


def cut_edges(edges, side) -> np.ndarray:
    edges = np.asarray(edges, dtype=np.int64)
    side = np.asarray(side)
    return np.array([e for e, (u, v) in enumerate(edges) if side[u] != side[v]], dtype=np.int64)


def mean_field_entropy(state, side) -> float:
    """Eq. apprx_entropy over the edges the bipartition cuts."""
    S = 0.0
    for e in cut_edges(state.edges, side):
        p = np.asarray(state.lam[e], dtype=np.float64) ** 2
        p = p[p > 0]
        S -= float(np.sum(p * np.log(p)))
    return S
