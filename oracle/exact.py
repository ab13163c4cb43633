"""Exact references for small systems — TEST INFRASTRUCTURE ONLY.

* State-vector dynamics of the same first-order Trotter circuit (App. F):
  the product of all edge gates of U_Z(t) is the diagonal exp(-i t E(z)) with
  E(z) = sum_e J_e z_u z_v + sum_a h_a z_a (each vertex receives D_a shares
  h_a/D_a), and U_X(t) = prod_a exp(-i t X_a).
* Contraction of a Vidal-gauge network to its state vector (Eq. vidal_gauge_tn).
* Brute-force maximisation of the objective (Eq. objective_function).

Qubit a is axis a of a (2,)*n array; index 0 is |0>, i.e. z = +1 (Sec. III.A).
"""

from __future__ import annotations

import numpy as np


def ising_diagonal(n: int, edges: np.ndarray, J: np.ndarray, h: np.ndarray) -> np.ndarray:
    """E(z) for every basis state, as a (2,)*n array."""
    idx = np.arange(2 ** n, dtype=np.int64)
    z = np.empty((n, 2 ** n), dtype=np.float64)
    for a in range(n):
        bit = (idx >> (n - 1 - a)) & 1
        z[a] = 1.0 - 2.0 * bit
    E = np.zeros(2 ** n, dtype=np.float64)
    for e in range(edges.shape[0]):
        E += J[e] * z[edges[e, 0]] * z[edges[e, 1]]
    for a in range(n):
        E += h[a] * z[a]
    return E.reshape((2,) * n)


def plus_state(n: int) -> np.ndarray:
    return np.full((2,) * n, 2.0 ** (-n / 2), dtype=np.complex128)


def apply_z_layer(psi: np.ndarray, diag: np.ndarray, theta: float) -> np.ndarray:
    return psi * np.exp(-1j * theta * diag)


def apply_x_layer(psi: np.ndarray, theta: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    W = np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    n = psi.ndim
    for a in range(n):
        psi = np.moveaxis(np.tensordot(W, psi, axes=([1], [a])), 0, a)
    return psi


def rho_single(psi: np.ndarray, a: int) -> np.ndarray:
    """Reduced density matrix of qubit a, unit trace."""
    n = psi.ndim
    p = np.moveaxis(psi, a, 0).reshape(2, -1)
    r = p @ p.conj().T
    return r / np.trace(r).real


def all_rho(psi: np.ndarray) -> np.ndarray:
    return np.stack([rho_single(psi, a) for a in range(psi.ndim)])


def anneal_statevector(inst, T: float, dt: float, record: bool = True):
    """Exact Trotterised anneal: per step U_Z(dt*k/K) then U_X(dt*(K-k)/K).
    Returns the final state and, if `record`, the per-step single-qubit
    reduced density matrices [K, n, 2, 2]."""
    n = inst.n
    diag = ising_diagonal(n, np.asarray(inst.edges), inst.J, inst.h)
    psi = plus_state(n)
    K = int(round(T / dt))
    rhos = []
    for k in range(1, K + 1):
        psi = apply_z_layer(psi, diag, dt * k / K)
        psi = apply_x_layer(psi, dt * (K - k) / K)
        if record:
            rhos.append(all_rho(psi))
    return psi, (np.stack(rhos) if record else None)


def evolve_product_formula(inst, theta_z, theta_x, theta_x0: float = 0.0) -> np.ndarray:
    """Exact state vector of any product formula built from the two layers:
    U_X(theta_x0) first, then per step U_Z(theta_z[k]) followed by
    U_X(theta_x[k]) (the first-order circuit of App. F has theta_x0 = 0; the
    symmetric second-order one merges the half mixing layers of adjacent
    steps).  The angles are inputs."""
    n = inst.n
    diag = ising_diagonal(n, np.asarray(inst.edges), inst.J, inst.h)
    psi = apply_x_layer(plus_state(n), theta_x0) if theta_x0 != 0.0 else plus_state(n)
    for tz, tx in zip(theta_z, theta_x):
        psi = apply_x_layer(apply_z_layer(psi, diag, tz), tx)
    return psi


def contract_network(state) -> np.ndarray:
    """Psi[i_1..i_n] = sum_j prod_a Gamma_a[i_a, j_da] prod_e lambda_e[j_e].

    Vertices are absorbed one at a time in index order; lambda_e is put on the
    vertex u of e = (u, v).  The running tensor carries the physical legs of
    the absorbed vertices and the bonds that still point outside."""
    n = state.n
    psi = np.ones((), dtype=np.complex128)
    phys = 0            # number of physical axes at the front of psi
    open_bonds = []     # bond (edge) ids of the remaining axes, in order
    for a in range(n):
        G = state.gamma[a]
        for k, e in enumerate(state.inc[a]):
            if int(state.edges[e, 0]) == a:
                shape = [1] * G.ndim
                shape[1 + k] = state.lam[e].shape[0]
                G = G * state.lam[e].reshape(shape)
        legs = list(state.inc[a])
        shared = [e for e in legs if e in open_bonds]
        ax_psi = [phys + open_bonds.index(e) for e in shared]
        ax_g = [1 + legs.index(e) for e in shared]
        psi = np.tensordot(psi, G, axes=(ax_psi, ax_g))
        # axes now: psi's remaining [phys..., open minus shared...] + G's [i_a, legs minus shared]
        rest_open = [e for e in open_bonds if e not in shared]
        new_open = [e for e in legs if e not in shared]
        # move i_a next to the other physical axes
        src = phys + len(rest_open)
        psi = np.moveaxis(psi, src, phys)
        phys += 1
        open_bonds = rest_open + new_open
    assert not open_bonds
    return psi


def normalised(psi: np.ndarray) -> np.ndarray:
    return psi / np.linalg.norm(psi)


def state_infidelity(psi: np.ndarray, phi: np.ndarray) -> float:
    """1 - |<psi|phi>|^2 for normalised inputs."""
    a = normalised(psi).ravel()
    b = normalised(phi).ravel()
    return float(1.0 - abs(np.vdot(a, b)) ** 2)


def brute_force_max(inst):
    """argmax_x E(x) over {-1,+1}^n and the maximum (exact for grid couplings)."""
    n = inst.n
    diag = ising_diagonal(n, np.asarray(inst.edges), inst.J, inst.h).ravel()
    k = int(np.argmax(diag))
    x = np.array([1 - 2 * ((k >> (n - 1 - a)) & 1) for a in range(n)], dtype=np.int8)
    return x, float(diag[k])


def trace_distance(r1: np.ndarray, r2: np.ndarray) -> float:
    return float(np.sum(np.abs(np.linalg.eigvalsh(r1 - r2))))


def mean_error(rho_exact: np.ndarray, rho_bp: np.ndarray, T: float, dt: float) -> float:
    """Eq. error: (dt / 2TN) sum_a sum_k ||rho_exact - rho_bp||_1."""
    K, n = rho_exact.shape[0], rho_exact.shape[1]
    tot = 0.0
    for k in range(K):
        for a in range(n):
            tot += trace_distance(rho_exact[k, a], rho_bp[k, a])
    return dt / (2.0 * T * n) * tot
