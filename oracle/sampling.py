"""BP-guided measurement sampling (Sec. IV.A, Eq. projection).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Qubits are measured one at a time, in ascending vertex order (reading: the
paper does not fix the order).  For qubit a: (i) rho_a from the BP messages
(Eq. partial_dens with Eq. bp_approx) of the last re-gauging, i.e. in the
symmetric gauge those messages were computed for; the outcome is x_a = +1
with probability rho_a[0, 0] and -1 otherwise, decided by a uniform number
u_a in [0, 1) supplied by the caller: x_a = +1 iff u_a < rho_a[0, 0];
(ii) the projector onto the outcome acts on Gamma_a's physical index
(Eq. projection); (iii) the network is re-gauged (symmetric gauge, BP from
the warm-start messages with the caller's tolerance and sweep cap, Alg. 2),
which also gives the messages for the next qubit.  One re-gauging before
the first qubit supplies its messages.
"""

from __future__ import annotations

import numpy as np

from . import gtqa as G


def sample(state: G.State, u, tol: float, max_sweeps: int):
    """Returns (x [n] int8, probability of each chosen outcome [n],
    residual R after each re-gauging [n], BP sweeps of each re-gauging [n])."""
    n = state.n
    u = np.asarray(u, dtype=np.float64)
    x = np.zeros(n, dtype=np.int8)
    prob = np.zeros(n)
    res = np.zeros(n)
    sweeps = np.zeros(n, dtype=np.int64)
    saved = (state.opts.bp_tol, state.opts.bp_max_sweeps)
    state.opts.bp_tol, state.opts.bp_max_sweeps = tol, max_sweeps

    def regauge_keep():
        T = G.symmetric_gauge(state)
        msgs = G.warm_messages(state)
        s, _ = G.belief_propagation(state, T, msgs, tol, max_sweeps, state.opts.bp_schedule)
        G.vidal_from_messages(state, T, msgs)
        return T, msgs, s

    try:
        T, msgs, _ = regauge_keep()
        for a in range(n):
            rho = G.rho_messages(state, T, msgs)[a]
            p0 = float(rho[0, 0].real)
            x[a] = 1 if u[a] < p0 else -1
            prob[a] = p0 if x[a] == 1 else 1.0 - p0
            keep = 0 if x[a] == 1 else 1          # |0> carries Z = +1
            Ga = state.gamma[a].copy()
            Ga[1 - keep] = 0.0
            state.gamma[a] = Ga
            T, msgs, sweeps[a] = regauge_keep()
            res[a] = G.vidal_residual(state)
    finally:
        state.opts.bp_tol, state.opts.bp_max_sweeps = saved
    return x, prob, res, sweeps
