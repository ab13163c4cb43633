"""Pins for the seeded inputs and the oracle's edge colouring (CPU only)."""

import numpy as np
import pytest

from oracle.colouring import check_colouring, misra_gries
from synthetic import (SplitMix64, grid_coupling, instance_from_edges,
                       random_regular_instance, random_tree_instance, schedule_angles)


def test_splitmix64_reference_sequence():
    # Published outputs of the reference splitmix64.c for seed 1234567.
    r = SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_bounded_is_uniform_and_in_range():
    r = SplitMix64(7)
    xs = [r.bounded(6) for _ in range(60000)]
    counts = np.bincount(xs, minlength=6)
    assert counts.min() > 9500 and counts.max() < 10500
    assert max(xs) == 5 and min(xs) == 0


def test_grid_coupling_range_and_grid():
    assert grid_coupling(0) == -1.0
    assert grid_coupling((1 << 64) - 1) == 1.0 - 2.0 ** -24
    r = SplitMix64(3)
    for _ in range(1000):
        x = r.grid_unit()
        assert -1.0 <= x < 1.0
        assert (x * 2 ** 24) == int(x * 2 ** 24)


@pytest.mark.parametrize("n", [4, 16, 100, 1000])
def test_random_regular_graph_invariants(n):
    inst = random_regular_instance(11 + n, n)
    e = inst.edges
    assert e.shape == (3 * n // 2, 2)
    assert (e[:, 0] < e[:, 1]).all()
    assert len({tuple(x) for x in e.tolist()}) == e.shape[0]          # simple
    assert sorted(map(tuple, e.tolist())) == list(map(tuple, e.tolist()))
    assert (inst.degrees() == 3).all()
    again = random_regular_instance(11 + n, n)
    assert np.array_equal(again.edges, e) and np.array_equal(again.J, inst.J)
    assert np.array_equal(again.h, inst.h)


def test_odd_n_rejected():
    with pytest.raises(ValueError):
        random_regular_instance(0, 15)


def test_tree_instance_is_a_tree():
    inst = random_tree_instance(5, 40)
    assert inst.n_edges == 39
    assert inst.degrees().max() <= 3
    # connected: union-find
    parent = list(range(inst.n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for u, v in inst.edges.tolist():
        parent[find(u)] = find(v)
    assert len({find(a) for a in range(inst.n)}) == 1


def test_energy_sums_exact_on_grid():
    # every partial sum of grid couplings is exact in binary64: order does not matter
    inst = random_regular_instance(2, 1000)
    x = np.where(np.arange(1000) % 3 == 0, 1.0, -1.0)
    terms = np.concatenate([inst.J * x[inst.edges[:, 0]] * x[inst.edges[:, 1]], inst.h * x])
    s1 = 0.0
    for t in terms:
        s1 += t
    s2 = 0.0
    for t in terms[::-1]:
        s2 += t
    s3 = float(np.sum(np.sort(terms)))
    assert s1 == s2 == s3


def test_schedule_angles():
    tz, tx = schedule_angles(10.0, 0.1)
    assert tz.size == 100
    assert tz[-1] == pytest.approx(0.1) and tx[-1] == 0.0
    assert tx[0] == pytest.approx(0.1 * 99 / 100)
    np.testing.assert_allclose(tz + tx, 0.1, rtol=0, atol=1e-16)


def _brute_force_chromatic_index_at_most(n, edges, k):
    """Small exhaustive search: is there a proper edge colouring with k colours?"""
    m = len(edges)
    col = [-1] * m

    def ok(e, c):
        u, v = edges[e]
        for f in range(e):
            if col[f] == c and (u in edges[f] or v in edges[f]):
                return False
        return True

    def rec(e):
        if e == m:
            return True
        for c in range(k):
            if ok(e, c):
                col[e] = c
                if rec(e + 1):
                    return True
                col[e] = -1
        return False
    return rec(0)


@pytest.mark.parametrize("seed", range(20))
def test_misra_gries_proper_and_at_most_delta_plus_one(seed):
    for n in (8, 16, 50, 200):
        inst = random_regular_instance(1000 * seed + n, n)
        col = misra_gries(inst.n, inst.edges)
        check_colouring(inst.n, inst.edges, col)
        assert col.max() <= 3
        # each colour class is a matching
        for c in range(col.max() + 1):
            vs = inst.edges[col == c].ravel()
            assert len(set(vs.tolist())) == vs.size


def test_misra_gries_special_graphs():
    # K4 (class 1: 3 colours suffice), Petersen graph (class 2: needs 4)
    k4 = instance_from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
    col = misra_gries(4, k4.edges)
    check_colouring(4, k4.edges, col)
    assert col.max() <= 3
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    pet = instance_from_edges(10, outer + spokes + inner)
    col = misra_gries(10, pet.edges)
    check_colouring(10, pet.edges, col)
    assert col.max() == 3
    assert not _brute_force_chromatic_index_at_most(10, [tuple(x) for x in pet.edges.tolist()], 3)
    tree = random_tree_instance(9, 30)
    col = misra_gries(30, tree.edges)
    check_colouring(30, tree.edges, col)
    assert col.max() <= 3


def test_misra_gries_is_deterministic():
    inst = random_regular_instance(99, 300)
    a = misra_gries(inst.n, inst.edges)
    b = misra_gries(inst.n, inst.edges.copy())
    assert np.array_equal(a, b)


def test_randomised_schedule_edge_cases():
    from synthetic import schedule_angles_randomised
    T, dt = 1.0, 0.25
    K = 4
    s = (np.arange(1, K + 1) - 0.5) / K
    ax = dt * (1 - s)
    with pytest.raises(ValueError):
        schedule_angles_randomised(T, dt, np.zeros(K - 1, dtype=bool))
    # every step interaction first: the plain midpoint steps, no leading layer
    tz, tx, tx0 = schedule_angles_randomised(T, dt, np.zeros(K, dtype=bool))
    assert tx0 == 0.0
    np.testing.assert_array_equal(tz, dt * s)
    np.testing.assert_array_equal(tx, ax)
    # every step mixing first: each mixing layer moves to the step before
    tz, tx, tx0 = schedule_angles_randomised(T, dt, np.ones(K, dtype=bool))
    assert tx0 == ax[0]
    np.testing.assert_array_equal(tx[:-1], ax[1:])
    assert tx[-1] == 0.0
