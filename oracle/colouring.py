"""Misra-Gries proper edge colouring with pinned tie-breaks (oracle side).

The paper applies the interaction layer U_Z gate by gate (App. F) and does not
say in which order; the engine groups the gates into colour classes (each a
matching) and applies the classes in colour-id order.  Misra and Gries' 1992
constructive proof of Vizing's theorem gives at most Delta+1 colours.  The
deterministic choices are:

* edges are coloured in edge-id order; for edge (u, v) with u < v the fan is
  built at u, starting from v;
* the fan is extended by scanning u's neighbours in ascending vertex id and
  taking the first w not yet in the fan whose edge (u, w) is coloured with a
  colour free at the current last fan vertex; repeat until no such w exists;
* c = lowest colour free at u, d = lowest colour free at the last fan vertex;
* the alternating path starting at u with colours d, c, d, ... is inverted;
* w = the first fan vertex (in fan order) such that the fan prefix ending at w
  is still a fan and d is free at w; the prefix is rotated and (u, w) gets d.

Pinned by tests: proper colouring, <= Delta+1 colours, each class a matching;
bit-exact agreement with the library's own implementation.
"""

from __future__ import annotations

import numpy as np


def misra_gries(n: int, edges: np.ndarray) -> np.ndarray:
    edges = np.asarray(edges)
    m = edges.shape[0]
    adj = [[] for _ in range(n)]          # (neighbour, edge id)
    for e in range(m):
        u, v = int(edges[e, 0]), int(edges[e, 1])
        adj[u].append((v, e))
        adj[v].append((u, e))
    for a in range(n):
        adj[a].sort()
    delta = max((len(x) for x in adj), default=0)
    ncol = delta + 1
    colour = [-1] * m
    # at[x][c] = edge id of colour c at vertex x, or -1
    at = [[-1] * ncol for _ in range(n)]

    def other(e, x):
        a, b = int(edges[e, 0]), int(edges[e, 1])
        return b if x == a else a

    def edge_id(x, y):
        for (w, e) in adj[x]:
            if w == y:
                return e
        raise KeyError((x, y))

    def is_free(x, c):
        return at[x][c] < 0

    def set_colour(e, c):
        a, b = int(edges[e, 0]), int(edges[e, 1])
        old = colour[e]
        if old >= 0:
            at[a][old] = -1
            at[b][old] = -1
        colour[e] = c
        if c >= 0:
            at[a][c] = e
            at[b][c] = e

    def lowest_free(x):
        for c in range(ncol):
            if is_free(x, c):
                return c
        raise RuntimeError("no free colour")

    for e0 in range(m):
        u, v = int(edges[e0, 0]), int(edges[e0, 1])
        # maximal fan at u starting at v
        fan = [v]
        in_fan = {v}
        while True:
            last = fan[-1]
            nxt = -1
            for (w, e) in adj[u]:
                if w in in_fan:
                    continue
                c = colour[e]
                if c >= 0 and is_free(last, c):
                    nxt = w
                    break
            if nxt < 0:
                break
            fan.append(nxt)
            in_fan.add(nxt)
        c = lowest_free(u)
        d = lowest_free(fan[-1])
        # invert the cd-path starting at u (first edge coloured d)
        if c != d:
            path = []
            x, want = u, d
            while True:
                e = at[x][want]
                if e < 0:
                    break
                path.append(e)
                x = other(e, x)
                want = c if want == d else d
            for e in path:
                set_colour(e, -1)
            # re-colour after clearing so that the at-tables stay consistent
            for idx, e in enumerate(path):
                set_colour(e, c if idx % 2 == 0 else d)
        # first fan vertex w such that the prefix up to w is a fan and d is free at w
        k = -1
        for i, w in enumerate(fan):
            if i > 0:
                ce = colour[edge_id(u, w)]
                if ce < 0 or not is_free(fan[i - 1], ce):
                    break
            if is_free(w, d):
                k = i
                break
        if k < 0:
            raise RuntimeError("Misra-Gries invariant violated")
        # rotate the fan prefix fan[0..k]
        for i in range(k):
            e_i = edge_id(u, fan[i])
            e_n = edge_id(u, fan[i + 1])
            cn = colour[e_n]
            set_colour(e_n, -1)
            set_colour(e_i, cn)
        set_colour(edge_id(u, fan[k]), d)
    return np.asarray(colour, dtype=np.int32)


def check_colouring(n: int, edges: np.ndarray, colour: np.ndarray) -> None:
    """Raise if `colour` is not a proper edge colouring."""
    seen = {}
    for e in range(edges.shape[0]):
        c = int(colour[e])
        if c < 0:
            raise AssertionError(f"edge {e} uncoloured")
        for x in (int(edges[e, 0]), int(edges[e, 1])):
            if (x, c) in seen:
                raise AssertionError(f"colour {c} repeated at vertex {x}")
            seen[(x, c)] = e
