"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
state-vector dynamics built from Kronecker products, the Schmidt
decomposition of the exact state across a tree edge, closed forms for product
states, brute force over all bit strings, and the paper's error band.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import exact as X
from oracle import gtqa as G
from synthetic import (instance_from_edges, random_regular_instance,
                       random_tree_instance, schedule_angles, schedule_angles_second_order,
                       schedule_angles_randomised)

PAULI_X = np.array([[0, 1], [1, 0]], dtype=complex)
PAULI_Z = np.diag([1.0, -1.0]).astype(complex)


def _kron_op(n, ops):
    """Tensor product with ops[a] on qubit a (identity elsewhere); qubit 0 leftmost."""
    out = np.ones((1, 1), dtype=complex)
    for a in range(n):
        out = np.kron(out, ops.get(a, np.eye(2)))
    return out


def _ising_matrix(inst):
    n = inst.n
    H = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for e, (u, v) in enumerate(inst.edges.tolist()):
        H += inst.J[e] * _kron_op(n, {u: PAULI_Z, v: PAULI_Z})
    for a in range(n):
        H += inst.h[a] * _kron_op(n, {a: PAULI_Z})
    return H


# ---------------------------------------------------------------- gates

def test_x_gate_is_matrix_exponential():
    for th in (0.0, 0.1, 0.7, -1.3):
        np.testing.assert_allclose(G.x_gate(th), sla.expm(-1j * th * PAULI_X), atol=1e-15)


def test_zz_gate_is_matrix_exponential():
    J, hu, hv, th = 0.37, -0.81, 0.22, 0.61
    H = J * np.kron(PAULI_Z, PAULI_Z) + hu * np.kron(PAULI_Z, np.eye(2)) + hv * np.kron(np.eye(2), PAULI_Z)
    W = G.zz_gate(th, J, hu, hv).reshape(4, 4)
    np.testing.assert_allclose(W, sla.expm(-1j * th * H), atol=1e-15)


def test_product_of_edge_gates_is_ising_evolution():
    inst = random_regular_instance(4, 6)
    st = G.init_state(inst)
    th = 0.43
    U = np.eye(2 ** 6, dtype=complex)
    for e, (u, v) in enumerate(inst.edges.tolist()):
        W = G.zz_gate(th, inst.J[e], inst.h[u] / st.deg[u], inst.h[v] / st.deg[v])
        d = np.array([W[iu, iv, iu, iv] for iu in range(2) for iv in range(2)])
        # embed the diagonal two-qubit gate
        ops = np.zeros(2 ** 6, dtype=complex)
        for k in range(2 ** 6):
            iu = (k >> (5 - u)) & 1
            iv = (k >> (5 - v)) & 1
            ops[k] = d[2 * iu + iv]
        U = U @ np.diag(ops)
    np.testing.assert_allclose(U, sla.expm(-1j * th * _ising_matrix(inst)), atol=1e-13)
    # and the state-vector reference uses the same diagonal
    diag = X.ising_diagonal(6, inst.edges, inst.J, inst.h).ravel()
    np.testing.assert_allclose(np.diag(_ising_matrix(inst)).real, diag, atol=1e-13)


def test_statevector_reference_matches_dense_expm():
    inst = random_regular_instance(8, 6)
    H = _ising_matrix(inst)
    Hx = sum(_kron_op(6, {a: PAULI_X}) for a in range(6))
    psi = np.full(2 ** 6, 2 ** -3, dtype=complex)
    psi_ref = X.plus_state(6)
    tz, tx = schedule_angles(1.0, 0.25)
    for k in range(tz.size):
        psi = sla.expm(-1j * tx[k] * Hx) @ (sla.expm(-1j * tz[k] * H) @ psi)
        psi_ref = X.apply_x_layer(X.apply_z_layer(psi_ref, X.ising_diagonal(6, inst.edges, inst.J, inst.h), tz[k]), tx[k])
    np.testing.assert_allclose(psi_ref.ravel(), psi, atol=1e-13)


# ---------------------------------------------------------------- exactness without truncation

@pytest.mark.parametrize("policy", ["never", "colour", "step"])
def test_untruncated_evolution_is_exact_on_loopy_graph(policy):
    inst = random_regular_instance(5, 10)
    st = G.init_state(inst, G.Options(chi=64, regauge=policy))
    diag = X.ising_diagonal(10, inst.edges, inst.J, inst.h)
    psi = X.plus_state(10)
    tz, tx = schedule_angles(2.0, 0.5)
    for k in range(2):
        G.trotter_step(st, tz[k], tx[k])
        psi = X.apply_x_layer(X.apply_z_layer(psi, diag, tz[k]), tx[k])
        assert X.state_infidelity(psi, X.contract_network(st)) < 1e-12


def test_untruncated_evolution_is_exact_on_tree_and_bp_is_exact():
    inst = random_tree_instance(3, 12)
    st = G.init_state(inst, G.Options(chi=64))
    diag = X.ising_diagonal(12, inst.edges, inst.J, inst.h)
    psi = X.plus_state(12)
    tz, tx = schedule_angles(2.0, 0.25)
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
        psi = X.apply_x_layer(X.apply_z_layer(psi, diag, tz[k]), tx[k])
    assert X.state_infidelity(psi, X.contract_network(st)) < 1e-12
    exact_rho = X.all_rho(psi)
    np.testing.assert_allclose(G.rho_vidal(st), exact_rho, atol=1e-12)
    # BP from random messages on a tree gives exact environments (Sec. II.B)
    T = G.symmetric_gauge(st)
    rng = np.random.default_rng(0)
    ent = [[rng.uniform(-1, 1, (st.lam[e].size,) * 2) + 1j * rng.uniform(-1, 1, (st.lam[e].size,) * 2)
            for _ in range(2)] for e in range(st.n_edges)]
    msgs = G.random_messages(st, ent)
    sweeps, dist = G.belief_propagation(st, T, msgs, 1e-14, 100)
    assert sweeps < 100
    np.testing.assert_allclose(G.rho_messages(st, T, msgs), exact_rho, atol=1e-12)
    # the flooding schedule from the same start reaches the same exact
    # environments; a flooding sweep is independent of the edge order, so
    # one sweep over the edges in reverse order gives the same messages
    msgs_f = G.random_messages(st, ent)
    sweeps_f, _ = G.belief_propagation(st, T, msgs_f, 1e-14, 100, "flooding")
    assert sweeps_f < 100
    np.testing.assert_allclose(G.rho_messages(st, T, msgs_f), exact_rho, atol=1e-12)
    one = G.random_messages(st, ent)
    G.belief_propagation(st, T, one, 0.0, 1, "flooding")
    rev = [[G.message_update(T[int(st.edges[e, sd])], int(st.legpos[e, sd]),
                             {k: G.incoming(st, G.random_messages(st, ent), int(st.edges[e, sd]), e2)
                              for k, e2 in enumerate(st.inc[int(st.edges[e, sd])]) if k != int(st.legpos[e, sd])})
            for sd in range(2)] for e in reversed(range(st.n_edges))]
    for i, e in enumerate(reversed(range(st.n_edges))):
        for sd in range(2):
            np.testing.assert_allclose(one[e][sd], rev[i][sd] / np.trace(rev[i][sd]), atol=1e-13)
    for e in range(st.n_edges):
        for d in range(2):
            m = msgs[e][d]
            np.testing.assert_allclose(m, m.conj().T, atol=1e-14)
            assert abs(np.trace(m) - 1) < 1e-14
            assert np.linalg.eigvalsh(m).min() > -1e-14


def _schmidt_values_across_edge(psi, inst, e):
    n = inst.n
    u, v = inst.edges[e]
    adj = {a: [] for a in range(n)}
    for f, (x, y) in enumerate(inst.edges.tolist()):
        if f != e:
            adj[x].append(y)
            adj[y].append(x)
    side = {int(u)}
    stack = [int(u)]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in side:
                side.add(y)
                stack.append(y)
    A = sorted(side)
    B = [a for a in range(n) if a not in side]
    M = np.transpose(psi, A + B).reshape(2 ** len(A), 2 ** len(B))
    s = np.linalg.svd(M / np.linalg.norm(M), compute_uv=False)
    return s


def test_vidal_gauge_on_tree_gives_schmidt_values_and_zero_residual():
    inst = random_tree_instance(21, 10)
    st = G.init_state(inst, G.Options(chi=64, regauge="never"))
    diag = X.ising_diagonal(10, inst.edges, inst.J, inst.h)
    psi = X.plus_state(10)
    tz, tx = schedule_angles(1.5, 0.25)
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
        psi = X.apply_x_layer(X.apply_z_layer(psi, diag, tz[k]), tx[k])
    # break the gauge by a non-unitary local map, then re-gauge with Alg. 1 + Alg. 2
    rng = np.random.default_rng(1)
    for a in range(st.n):
        M = np.eye(2) + 0.3 * (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
        st.gamma[a] = np.tensordot(M, st.gamma[a], axes=([1], [0]))
        psi = np.moveaxis(np.tensordot(M, psi, axes=([1], [a])), 0, a)
    assert G.vidal_residual(st) > 1e-2
    st.opts.bp_tol = 1e-14
    st.opts.bp_max_sweeps = 200
    G.regauge(st)
    assert G.vidal_residual(st) < 1e-10
    assert X.state_infidelity(psi, X.contract_network(st)) < 1e-12
    for e in range(st.n_edges):
        s = _schmidt_values_across_edge(psi, inst, e)
        lam = st.lam[e]
        np.testing.assert_allclose(lam, s[:lam.size], atol=1e-10)
        assert np.sum(s[lam.size:] ** 2) < 1e-20


def test_regauge_is_a_gauge_transform_on_loopy_graph():
    inst = random_regular_instance(17, 10)
    st = G.init_state(inst, G.Options(chi=2, regauge="never"))
    tz, tx = schedule_angles(3.0, 0.5)
    for k in range(3):
        G.trotter_step(st, tz[k], tx[k])      # truncation breaks the gauge
    before = X.contract_network(st)
    r0 = G.vidal_residual(st)
    st.opts.chi = 64
    st.opts.bp_tol = 1e-13
    st.opts.bp_max_sweeps = 500
    sweeps, dist = G.regauge(st)
    assert dist < 1e-13
    after = X.contract_network(st)
    assert X.state_infidelity(before, after) < 1e-10
    assert G.vidal_residual(st) < 1e-8 < r0


def test_warm_start_messages_are_the_fixed_point():
    # Reading of Eq. reconstructed_messages: diag(lambda) is the BP fixed point
    # of T = Gamma lambda^(1/2) in exact Vidal gauge; the printed lambda^(1/2) is not.
    inst = random_tree_instance(6, 12)
    st = G.init_state(inst, G.Options(chi=64, regauge="never"))
    tz, tx = schedule_angles(1.0, 0.25)
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
    T = G.symmetric_gauge(st)
    sweeps, dist = G.belief_propagation(st, T, G.warm_messages(st), 1e-12, 1)
    assert dist < 1e-13
    st.opts.warm_start = "sqrt_lambda"
    sweeps, dist = G.belief_propagation(st, T, G.warm_messages(st), 1e-12, 1)
    assert dist > 1e-4


def test_truncation_error_is_eckart_young():
    inst = random_tree_instance(2, 10)
    st = G.init_state(inst, G.Options(chi=64, regauge="never"))
    tz, tx = schedule_angles(2.0, 0.25)
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
    psi = X.contract_network(st)
    e = int(np.argmax(st.bond_dims()))
    d = st.lam[e].size
    assert d >= 3
    eps = G.truncate_edge(st, e, d - 2)
    trunc = X.contract_network(st)
    assert abs(np.linalg.norm(psi - trunc) - eps) < 1e-12
    assert abs(eps - np.sqrt(np.sum(np.sort(_schmidt_values_across_edge(psi, inst, e))[::-1][d - 2:] ** 2))) < 1e-10


def test_simple_update_truncation_fidelity_on_tree():
    inst = random_tree_instance(31, 10)
    st = G.init_state(inst, G.Options(chi=64, regauge="never"))
    tz, tx = schedule_angles(3.0, 0.3)
    for k in range(tz.size - 1):
        G.trotter_step(st, tz[k], tx[k])
    diag = X.ising_diagonal(10, inst.edges, inst.J, inst.h)
    e = int(np.argmax(st.bond_dims()))
    psi = X.contract_network(st)
    u, v = st.edges[e]
    W = G.zz_gate(tz[-1], st.J[e], st.h[u] / st.deg[u], st.h[v] / st.deg[v])
    # exact action of the single gate on the state vector (u < v: axis order kept)
    Wd = np.array([[W[0, 0, 0, 0], W[0, 1, 0, 1]], [W[1, 0, 1, 0], W[1, 1, 1, 1]]])
    psi_g = psi * Wd.reshape([2 if a in (u, v) else 1 for a in range(10)])
    d_eff = int(np.count_nonzero(st.lam[e] > 1e-8))
    assert d_eff >= 3
    st.opts.chi = d_eff - 1                 # forces truncation
    f, eps = G.simple_update(st, e, tz[-1])
    trunc = X.contract_network(st)
    infid = X.state_infidelity(psi_g, trunc)
    assert eps > 1e-8
    assert abs(infid - eps ** 2) < 1e-10
    assert abs(f - (1 - eps ** 2) ** 2) < 1e-12


# ---------------------------------------------------------------- product-state closed forms

def _single_qubit_closed_form(h, tz, tx):
    """<Z> of |+> under prod_k exp(-i tx_k X) exp(-i tz_k h Z)."""
    psi = np.array([1, 1], dtype=complex) / np.sqrt(2)
    zs = []
    for a, b in zip(tz, tx):
        psi = np.array([np.exp(-1j * a * h), np.exp(1j * a * h)]) * psi
        psi = sla.expm(-1j * b * PAULI_X) @ psi
        zs.append(abs(psi[0]) ** 2 - abs(psi[1]) ** 2)
    return np.array(zs)


def test_zero_coupling_closed_form_at_n1000():
    inst = random_regular_instance(1000, 1000, couplings="zero-j")
    st = G.init_state(inst, G.Options(chi=4))
    tz, tx = schedule_angles(100.0, 0.05)
    steps = 3
    zs = []
    for k in range(steps):
        G.trotter_step(st, tz[k], tx[k])
        zs.append(G.readout(st)[0])
        assert st.bond_dims().max() == 1
    for a in range(0, 1000, 37):
        ref = _single_qubit_closed_form(inst.h[a], tz[:steps], tx[:steps])
        np.testing.assert_allclose([z[a] for z in zs], ref, atol=1e-13)


def test_first_colour_class_closed_form_at_n1000():
    inst = random_regular_instance(1000, 1000)
    st = G.init_state(inst, G.Options(chi=4))
    th = 0.3
    cls = st.classes[0]
    for e in cls:
        G.simple_update(st, e, th)
    G.regauge(st)
    rho = G.rho_vidal(st)
    covered = set()
    for e in cls:
        u, v = (int(x) for x in st.edges[e])
        covered |= {u, v}
        psi = np.full((2, 2), 0.5, dtype=complex)
        for iu in range(2):
            for iv in range(2):
                zu, zv = 1 - 2 * iu, 1 - 2 * iv
                psi[iu, iv] *= np.exp(-1j * th * (inst.J[e] * zu * zv + inst.h[u] / 3 * zu + inst.h[v] / 3 * zv))
        ru = psi @ psi.conj().T
        rv = psi.T @ psi.conj()
        np.testing.assert_allclose(rho[u], ru, atol=1e-12)
        np.testing.assert_allclose(rho[v], rv, atol=1e-12)
    for a in range(inst.n):
        if a not in covered:
            np.testing.assert_allclose(rho[a], np.full((2, 2), 0.5), atol=1e-12)


# ---------------------------------------------------------------- BP mechanics

def test_bp_fixed_sweep_mode_and_schedules_agree():
    inst = random_regular_instance(3, 16)
    st = G.init_state(inst, G.Options(chi=4, regauge="never"))
    tz, tx = schedule_angles(2.0, 0.1)
    for k in range(10):
        G.trotter_step(st, tz[k], tx[k])
    T = G.symmetric_gauge(st)
    m1 = G.warm_messages(st)
    s, d = G.belief_propagation(st, T, m1, 0.0, 7)
    assert s == 7
    m_col = G.warm_messages(st)
    m_fl = G.warm_messages(st)
    s1, d1 = G.belief_propagation(st, T, m_col, 1e-13, 400, "colour")
    s2, d2 = G.belief_propagation(st, T, m_fl, 1e-13, 400, "flooding")
    assert d1 < 1e-13 and d2 < 1e-13 and s1 <= s2
    np.testing.assert_allclose(G.rho_messages(st, T, m_col), G.rho_messages(st, T, m_fl), atol=1e-11)


def test_readout_from_messages_matches_vidal_after_regauge():
    inst = random_regular_instance(12, 16)
    st = G.init_state(inst, G.Options(chi=4))
    tz, tx = schedule_angles(2.0, 0.1)
    for k in range(8):
        G.trotter_step(st, tz[k], tx[k])
    T = G.symmetric_gauge(st)
    msgs = G.warm_messages(st)
    G.belief_propagation(st, T, msgs, 1e-12, 200)
    np.testing.assert_allclose(G.rho_messages(st, T, msgs), G.rho_vidal(st), atol=1e-5)


# ---------------------------------------------------------------- objective, rounding

def test_objective_and_rounding_against_brute_force():
    inst = random_regular_instance(44, 12)
    x, Emax = X.brute_force_max(inst)
    assert G.objective(inst.edges, inst.J, inst.h, x) == Emax
    diag = X.ising_diagonal(12, inst.edges, inst.J, inst.h).ravel()
    assert Emax == diag.max()
    # rounding rule on a basis state's density matrices returns that basis state
    rho = np.zeros((12, 2, 2), dtype=complex)
    for a in range(12):
        rho[a, 0, 0] = 1.0 if x[a] == 1 else 0.0
        rho[a, 1, 1] = 1.0 - rho[a, 0, 0]
    assert np.array_equal(G.rounding(rho), x)
    tie = np.array([[[0.5, 0], [0, 0.5]]], dtype=complex)
    assert G.rounding(tie)[0] == -1


# ---------------------------------------------------------------- the paper's accuracy band

@pytest.mark.parametrize("seed", [0, 1])
def test_mean_trace_distance_error_in_paper_band(seed):
    # Eq. error at chi=4 on 16-qubit random 3-regular graphs: the paper reports
    # per-graph means of 1e-3 .. a few 1e-2 (Sec. III.D, Fig. 4b).
    inst = random_regular_instance(seed, 16)
    T, dt = 4.0, 0.1
    st = G.init_state(inst, G.Options(chi=4))
    tz, tx = schedule_angles(T, dt)
    rhos = []
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
        rhos.append(G.rho_vidal(st))
    _, rex = X.anneal_statevector(inst, T, dt)
    err = X.mean_error(rex, np.stack(rhos), T, dt)
    assert 1e-5 < err < 5e-2


def test_mean_error_closed_forms():
    # Eq. error, (dt / 2TN) sum_k sum_a ||rho_exact - rho||_1 over K = T/dt
    # steps: orthogonal pure states (trace distance 2 everywhere) give exactly
    # 1; diag(3/4, 1/4) against |0><0| (trace distance 1/2) gives 1/4; equal
    # states give 0; one qubit of N differing at one step of K gives 2/(2NK) * ...
    T, dt, n = 2.0, 0.25, 3
    K = int(round(T / dt))
    zero = np.array([[1, 0], [0, 0]], dtype=complex)
    one = np.array([[0, 0], [0, 1]], dtype=complex)
    mixed = np.diag([0.75, 0.25]).astype(complex)
    ex = np.tile(zero, (K, n, 1, 1))
    assert X.mean_error(ex, np.tile(one, (K, n, 1, 1)), T, dt) == pytest.approx(1.0, abs=1e-15)
    assert X.mean_error(ex, np.tile(mixed, (K, n, 1, 1)), T, dt) == pytest.approx(0.25, abs=1e-15)
    assert X.mean_error(ex, ex.copy(), T, dt) == 0.0
    single = ex.copy()
    single[3, 1] = one
    assert X.mean_error(ex, single, T, dt) == pytest.approx(dt / (2 * T * n) * 2.0, abs=1e-15)


def test_anneal_is_the_statevector_anneal_when_untruncated():
    # anneal(): App. F's first-order circuit with s(t) = 1 - t/T from |+>^N;
    # untruncated (chi above every bond's rank) on a tree, where the Vidal-form
    # readout is exact, it must reproduce the exact state-vector anneal at
    # every step, and its checkpoints are readouts of those steps
    inst = random_tree_instance(6, 8)
    T, dt = 1.2, 0.2
    st, out = G.anneal(inst, T, dt, G.Options(chi=16, bp_tol=1e-13, bp_max_sweeps=200), record_z=True,
                       checkpoints=(1, 3, 6))
    _, rex = X.anneal_statevector(inst, T, dt)
    zex = (rex[:, :, 0, 0] - rex[:, :, 1, 1]).real
    assert len(out["z"]) == 6
    np.testing.assert_allclose(np.stack(out["z"]), zex, atol=1e-10)
    for k, c in out["checkpoints"].items():
        np.testing.assert_allclose(c["z"], zex[k - 1], atol=1e-10)
        assert c["E"] == G.objective(inst.edges, inst.J, inst.h, c["x"])
    # the callback sees each checkpoint once, in order, after its readout
    seen = []
    G.anneal(inst, T, dt, G.Options(chi=16), checkpoints=(2, 5),
             on_checkpoint=lambda k, o, s_: seen.append((k, sorted(o["checkpoints"]))))
    assert seen == [(2, [2]), (5, [2, 5])]


def test_residual_closed_form_on_one_edge():
    # one edge: M_{a->b} = Gamma_a Gamma_a^dagger over the physical index;
    # Gamma_0 = [[1,1],[0,1]] gives M = [[1,1],[1,2]], eigenvalues (3 +- sqrt5)/2,
    # after division by tr M / 2 those of 1 - M are -+ sqrt5/3: trace norm 2 sqrt5/3.
    inst = instance_from_edges(2, [(0, 1)])
    st = G.init_state(inst, G.Options(chi=2))
    st.lam[0] = np.array([0.8, 0.6])
    st.gamma[0] = np.array([[1.0, 1.0], [0.0, 1.0]], dtype=complex)
    st.gamma[1] = 7.0 * np.eye(2, dtype=complex)          # orthogonal up to scale: no term
    assert G.vidal_residual(st) == pytest.approx((2 * np.sqrt(5) / 3) / 2, rel=1e-14)
    st.gamma[0] = np.diag([1.0, 2.0]).astype(complex)     # diag(0.4, 1.6): 1.2
    assert G.vidal_residual(st) == pytest.approx(0.6, rel=1e-14)
    st.gamma[0] = st.gamma[0] * (2.5 - 1j)               # scale-free
    assert G.vidal_residual(st) == pytest.approx(0.6, rel=1e-14)


def test_adaptive_policy_limits():
    # res_max < 0 re-gauges after every class (= "colour"); res_max = inf never does
    inst = random_regular_instance(41, 10)
    tz, tx = schedule_angles(4.0, 0.4)
    runs = {}
    for name, kw in (("colour", dict(regauge="colour")),
                     ("adapt_always", dict(regauge="adaptive", res_max=-1.0)),
                     ("never", dict(regauge="never")),
                     ("adapt_never", dict(regauge="adaptive", res_max=np.inf))):
        st = G.init_state(inst, G.Options(chi=2, bp_tol=0.0, bp_max_sweeps=5, **kw))
        for k in range(4):
            G.trotter_step(st, tz[k], tx[k])
        runs[name] = st
    for a, b in (("colour", "adapt_always"), ("never", "adapt_never")):
        for x, y in zip(runs[a].gamma, runs[b].gamma):
            assert np.array_equal(x, y)
        for x, y in zip(runs[a].lam, runs[b].lam):
            assert np.array_equal(x, y)


def test_adaptive_policy_regauges_when_residual_exceeds_threshold():
    inst = random_regular_instance(43, 12)
    tz, tx = schedule_angles(6.0, 0.3)
    st = G.init_state(inst, G.Options(chi=2, bp_tol=1e-12, bp_max_sweeps=200,
                                      regauge="adaptive", res_max=1e-5))
    n_reg = 0
    n_cls = 0
    for k in range(12):
        ss = G.trotter_step(st, tz[k], tx[k])
        n_cls += len(ss.residuals)
        n_reg += len(ss.sweeps)
        assert len(ss.sweeps) == sum(r > 1e-5 for r in ss.residuals)
    assert 0 < n_reg < n_cls
    # after a re-gauge the network is back in Vidal gauge
    G.regauge(st)
    assert G.vidal_residual(st) < 1e-8


def test_bp_stays_at_the_fixed_point_over_many_sweeps():
    # Unit trace (App. B) is imposed with the complex trace: a complex scale
    # left on a message would be compounded by the multilinear update of
    # Alg. 1, and the messages would drift off the fixed point and lose
    # Hermiticity as the sweeps go on.
    inst = random_regular_instance(0, 16)
    tz, tx = schedule_angles(10.0, 0.1)
    st = G.init_state(inst, G.Options(chi=4, bp_tol=0.0, bp_max_sweeps=6))
    for k in range(3):
        G.trotter_step(st, tz[k], tx[k])
    T = G.symmetric_gauge(st)
    msgs = G.warm_messages(st)
    _, dist = G.belief_propagation(st, T, msgs, 0.0, 80)
    assert dist < 1e-14
    for pair in msgs:
        for m in pair:
            assert np.max(np.abs(m - m.conj().T)) < 1e-14
            assert abs(np.trace(m) - 1.0) < 1e-14


# ---------------------------------------------------------------- entropy (Sec. III.C)

def _dumbbell():
    # two K4s, each missing one edge, joined by a bridge: the ratio cut of
    # Eq. bipartition is the bridge (1 / (4 * 4)), and no other cut reaches it
    e = [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 6), (4, 7), (5, 6), (5, 7), (6, 7), (0, 4)]
    return 8, sorted((min(u, v), max(u, v)) for u, v in e)


def test_spectral_bipartition_finds_the_bridge():
    from oracle import entropy as H
    n, edges = _dumbbell()
    side = H.spectral_bipartition(n, edges)
    assert set(np.flatnonzero(side)) in ({0, 1, 2, 3}, {4, 5, 6, 7})
    assert H.cut_ratio(n, edges, side) == 1 / 16
    # brute force over all 2^8 subsets: nothing beats it
    best = min(H.cut_ratio(n, edges, [(s >> a) & 1 for a in range(n)]) for s in range(1, 2 ** n - 1))
    assert best == 1 / 16


def test_spectral_bipartition_separates_weakly_joined_halves():
    from oracle import entropy as H
    a = random_regular_instance(7, 20)
    b = random_regular_instance(8, 20)
    # drop one edge in each half and join the freed endpoints across
    ea = [tuple(x) for x in a.edges.tolist()]
    eb = [tuple(x) for x in b.edges.tolist()]
    (u1, v1), (u2, v2) = ea.pop(0), eb.pop(0)
    edges = ea + [(u + 20, v + 20) for u, v in eb] + [(u1, u2 + 20), (v1, v2 + 20)]
    edges = sorted((min(u, v), max(u, v)) for u, v in edges)
    side = H.spectral_bipartition(40, edges)
    assert set(np.flatnonzero(side)) in (set(range(20)), set(range(20, 40)))
    assert len(H.cut_edges(edges, side)) == 2


def test_mean_field_entropy_closed_forms():
    from oracle import entropy as H
    inst = instance_from_edges(2, [(0, 1)])
    st = G.init_state(inst, G.Options(chi=2))
    assert H.mean_field_entropy(st, [0, 1]) == 0.0          # product state
    st.lam[0] = np.array([1.0, 1.0]) / np.sqrt(2.0)
    assert H.mean_field_entropy(st, [0, 1]) == pytest.approx(np.log(2.0), rel=1e-15)
    p = 0.3
    st.lam[0] = np.sqrt([1 - p, p])
    assert H.mean_field_entropy(st, [1, 0]) == pytest.approx(-(p * np.log(p) + (1 - p) * np.log(1 - p)),
                                                             rel=1e-14)
    assert H.mean_field_entropy(st, [1, 1]) == 0.0          # no cut edge


def test_mean_field_entropy_on_a_tree_cut_is_the_exact_entropy():
    # one cut edge of a tree in Vidal gauge: the lambdas are the exact Schmidt
    # values across it, so Eq. apprx_entropy is the exact entanglement entropy
    from oracle import entropy as H
    inst = random_tree_instance(21, 10)
    st = G.init_state(inst, G.Options(chi=64, regauge="never"))
    diag = X.ising_diagonal(10, inst.edges, inst.J, inst.h)
    psi = X.plus_state(10)
    tz, tx = schedule_angles(1.5, 0.25)
    for k in range(tz.size):
        G.trotter_step(st, tz[k], tx[k])
        psi = X.apply_x_layer(X.apply_z_layer(psi, diag, tz[k]), tx[k])
    for e in (0, 4, 8):
        s = _schmidt_values_across_edge(psi, inst, e)
        p = s ** 2
        p = p[p > 1e-30]
        exact = float(-np.sum(p * np.log(p)))
        # the side of the tree containing the edge's first endpoint
        u, v = inst.edges[e]
        comp = {int(u)}
        frontier = [int(u)]
        adj = {a: [] for a in range(10)}
        for f, (x, y) in enumerate(inst.edges.tolist()):
            if f != e:
                adj[x].append(y)
                adj[y].append(x)
        while frontier:
            a = frontier.pop()
            for b in adj[a]:
                if b not in comp:
                    comp.add(b)
                    frontier.append(b)
        side = [1 if a in comp else 0 for a in range(10)]
        assert list(H.cut_edges(inst.edges, side)) == [e]
        assert H.mean_field_entropy(st, side) == pytest.approx(exact, abs=1e-10)


# ---------------------------------------------------------------- sampling (Sec. IV.A)

def test_sampling_on_a_tree_draws_from_the_exact_distribution():
    # on a tree the re-gauged network is exact after every projection, so the
    # product of the chosen outcomes' probabilities is |psi(x)|^2.  With the
    # default cutoffs it is so to ~1e-8: a projection leaves rank-deficient
    # messages whose smallest eigenvalues the Alg. 2 cutoff (1e-14 of the
    # largest) drops; without cutoffs to ~1e-10.
    from oracle import sampling as SM
    inst = random_tree_instance(33, 8)
    diag = X.ising_diagonal(8, inst.edges, inst.J, inst.h)
    tz, tx = schedule_angles(1.5, 0.25)
    rng = np.random.default_rng(5)
    for trial in range(6):
        cuts = {} if trial < 3 else {"eig_cut": 0.0, "svd_cut": 0.0}
        rel = 1e-6 if trial < 3 else 1e-9
        st = G.init_state(inst, G.Options(chi=64, bp_tol=1e-13, bp_max_sweeps=500, **cuts))
        psi = X.plus_state(8)
        for k in range(tz.size):
            G.trotter_step(st, tz[k], tx[k])
            psi = X.apply_x_layer(X.apply_z_layer(psi, diag, tz[k]), tx[k])
        u = rng.random(8)
        x, prob, res, sweeps = SM.sample(st, u, 0.0 if trial >= 3 else 1e-13, 20 if trial >= 3 else 500)
        idx = tuple(0 if xa == 1 else 1 for xa in x)
        p_exact = abs(psi[idx]) ** 2 / np.sum(np.abs(psi) ** 2)
        assert np.prod(prob) == pytest.approx(p_exact, rel=rel)
        # the final network is the product state |x>
        z = G.readout(st)[0]
        np.testing.assert_allclose(z, x.astype(float), atol=1e-10)


def test_sampling_a_basis_state_is_deterministic():
    from oracle import sampling as SM
    inst = random_regular_instance(9, 10)
    st = G.init_state(inst, G.Options(chi=4))
    flip = [a for a in range(10) if a % 3 == 0]
    for a in range(10):      # |+> -> |0> or |1> by a pi/4 rotation about Y-free X path: set directly
        g = np.zeros_like(st.gamma[a])
        g[1 if a in flip else 0] = 1.0
        st.gamma[a] = g
    for u in (np.zeros(10), np.full(10, 0.999999)):
        s2 = G.init_state(inst, G.Options(chi=4))
        s2.gamma = [g.copy() for g in st.gamma]
        x, prob, _, _ = SM.sample(s2, u, 1e-12, 50)
        assert list(x) == [-1 if a in flip else 1 for a in range(10)]
        np.testing.assert_allclose(prob, 1.0, atol=1e-12)


# ---------------------------------------------------------------- product formulas (Sec. VI, App. F)

def _exact_anneal(inst, T):
    """Time-ordered evolution under H(t) = (1 - t/T) sum X + (t/T) H_Ising
    from |+>^n, integrated to 1e-13 (the limit dt -> 0 of both formulas)."""
    from scipy.integrate import solve_ivp
    n = inst.n
    Hz = np.diag(X.ising_diagonal(n, inst.edges, inst.J, inst.h).ravel()).astype(complex)
    Hx = sum(_kron_op(n, {a: PAULI_X}) for a in range(n))
    psi0 = X.plus_state(n).ravel()
    sol = solve_ivp(lambda t, y: -1j * (((1 - t / T) * Hx + (t / T) * Hz) @ y), (0.0, T), psi0,
                    method="DOP853", rtol=1e-13, atol=1e-13)
    return sol.y[:, -1]


def test_second_order_formula_converges_quadratically():
    # Trotter error against the exact time-ordered evolution: halving dt
    # halves it for the first-order circuit and quarters it for the
    # symmetric second-order one
    inst = random_regular_instance(3, 4)
    T = 2.0
    exact = _exact_anneal(inst, T)
    e1, e2 = [], []
    for dt in (0.1, 0.05, 0.025):
        tz, tx = schedule_angles(T, dt)
        e1.append(np.linalg.norm(X.evolve_product_formula(inst, tz, tx).ravel() - exact))
        tz2, tx2, tx0 = schedule_angles_second_order(T, dt)
        e2.append(np.linalg.norm(X.evolve_product_formula(inst, tz2, tx2, tx0).ravel() - exact))
    r1 = [e1[i] / e1[i + 1] for i in range(2)]
    r2 = [e2[i] / e2[i + 1] for i in range(2)]
    assert all(1.7 < r < 2.4 for r in r1), r1
    assert all(3.5 < r < 4.5 for r in r2), r2
    assert e2[-1] < 0.1 * e1[-1]


def test_second_order_angles_merge_the_half_layers():
    T, dt = 3.0, 0.5
    tz, tx, tx0 = schedule_angles_second_order(T, dt)
    K = 6
    s = (np.arange(1, K + 1) - 0.5) / K
    np.testing.assert_allclose(tz, dt * s, rtol=0, atol=1e-15)
    a = dt * (1 - s) / 2
    assert tx0 == a[0]
    np.testing.assert_allclose(tx[:-1], a[:-1] + a[1:], rtol=0, atol=1e-15)
    assert tx[-1] == a[-1]
    # the total mixing angle equals the midpoint rule for the mixing term
    np.testing.assert_allclose(tx0 + tx.sum(), dt * (1 - s).sum(), rtol=1e-14)


def test_untruncated_second_order_network_is_the_product_formula():
    inst = random_regular_instance(5, 8)
    tz, tx, tx0 = schedule_angles_second_order(1.0, 0.5)
    st, _ = G.run_angles(inst, tz, tx, tx0, G.Options(chi=64))
    psi = X.evolve_product_formula(inst, tz, tx, tx0)
    assert X.state_infidelity(psi, X.contract_network(st)) < 1e-12


def _layer_unitaries(inst):
    """Dense Z(theta) and X(theta) layers of the n-qubit circuit (closed forms:
    a diagonal phase exp(-i theta E(z)) and the tensor power of
    cos(theta) I - i sin(theta) X)."""
    n = inst.n
    diag = X.ising_diagonal(n, inst.edges, inst.J, inst.h).ravel()

    def uz(th):
        return np.diag(np.exp(-1j * th * diag))

    def ux(th):
        w = np.cos(th) * np.eye(2) - 1j * np.sin(th) * PAULI_X
        u = np.ones((1, 1), dtype=complex)
        for _ in range(n):
            u = np.kron(u, w)
        return u
    return uz, ux


def test_randomised_angles_follow_the_layer_order():
    # the merged (theta_z, theta_x, theta_x0) form applies exactly the drawn
    # layer sequence: per step X then Z when x_first, else Z then X
    inst = random_regular_instance(5, 4)
    T, dt = 2.0, 0.25
    K = 8
    uz, ux = _layer_unitaries(inst)
    for seed in range(4):
        xf = np.random.default_rng(seed).random(K) < 0.5
        xf[0] = seed % 2 == 0                  # both a leading and a trailing mixing layer occur
        tz, tx, tx0 = schedule_angles_randomised(T, dt, xf)
        psi = X.plus_state(inst.n).ravel()
        for k in range(K):
            s = (k + 0.5) / K
            a, b = ux(dt * (1 - s)), uz(dt * s)
            psi = (b @ (a @ psi)) if xf[k] else (a @ (b @ psi))
        got = X.evolve_product_formula(inst, tz, tx, tx0).ravel()
        np.testing.assert_allclose(got, psi, atol=1e-13)
        # every step's mixing angle is used once
        np.testing.assert_allclose(tx0 + tx.sum(), dt * (1 - (np.arange(K) + 0.5) / K).sum(), rtol=1e-14)


def test_randomised_formula_averages_to_second_order():
    # With fair coins the averaged channel (1/2)(XZ . ZX-conjugations) of each
    # step is second order in dt (the trace distance to the exact time-ordered
    # state quarters when dt halves), while a fixed order is first order.
    inst = random_regular_instance(3, 4)
    T = 2.0
    psi_ex = _exact_anneal(inst, T)
    rho_ex = np.outer(psi_ex, psi_ex.conj())
    uz, ux = _layer_unitaries(inst)
    er, ef = [], []
    for dt in (0.1, 0.05, 0.025):
        K = int(round(T / dt))
        p0 = X.plus_state(inst.n).ravel()
        rho = np.outer(p0, p0.conj())
        for k in range(K):
            s = (k + 0.5) / K
            A = ux(dt * (1 - s)) @ uz(dt * s)      # Z first
            B = uz(dt * s) @ ux(dt * (1 - s))      # X first
            rho = 0.5 * (A @ rho @ A.conj().T + B @ rho @ B.conj().T)
        er.append(X.trace_distance(rho, rho_ex))
        tz, tx, tx0 = schedule_angles_randomised(T, dt, np.zeros(K, dtype=bool))
        pf = X.evolve_product_formula(inst, tz, tx, tx0).ravel()
        ef.append(X.trace_distance(np.outer(pf, pf.conj()), rho_ex))
    rr = [er[i] / er[i + 1] for i in range(2)]
    rf = [ef[i] / ef[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.5 for r in rr), rr
    assert all(1.7 < r < 2.4 for r in rf), rf
    # and the average over every coin pattern of the merged form is that channel
    dt = 0.5
    K = 4
    p0 = X.plus_state(inst.n).ravel()
    rho = np.outer(p0, p0.conj())
    for k in range(K):
        s = (k + 0.5) / K
        A = ux(dt * (1 - s)) @ uz(dt * s)
        B = uz(dt * s) @ ux(dt * (1 - s))
        rho = 0.5 * (A @ rho @ A.conj().T + B @ rho @ B.conj().T)
    avg = np.zeros_like(rho)
    for pattern in range(2 ** K):
        xf = np.array([(pattern >> k) & 1 for k in range(K)], dtype=bool)
        pf = X.evolve_product_formula(inst, *schedule_angles_randomised(T, dt, xf)).ravel()
        avg += np.outer(pf, pf.conj()) / 2 ** K
    np.testing.assert_allclose(avg, rho, atol=1e-13)
