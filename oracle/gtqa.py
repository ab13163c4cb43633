"""Graph tensor-network quantum annealer (GTQA), plain complex128 NumPy oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function follows
the paper's definitions in the paper's order; LAPACK (numpy.linalg svd/eigh)
serves as the linear-algebra primitive.  Readings of silent or ambiguous
points are named where they are used:

* step order: within Trotter step k the interaction layer U_Z(dt*(1-s_k))
  acts first, then the mixing layer U_X(dt*s_k), s_k = s(k dt) = 1 - k/K
  (App. F, Eq. discretizatoion, read as a time-ordered product);
* U_Z is applied colour class by colour class in colour-id order (App. F
  leaves the gate order open); a class is a matching, so gates inside it
  commute and touch disjoint tensors;
* gates: exp(-i t X) and exp(-i t (J Z Z + h_a/D_a Z_a + h_b/D_b Z_b)) with no
  factor 1/2, D_a the degree of a, Z|0> = +|0> (App. F, Sec. III.A);
* truncation keeps r = min(chi, #{sigma_k > svd_cut * sigma_0}) singular
  values (Alg. 3 plus a relative cutoff for exactly/numerically zero ones);
  kept values are renormalised to unit 2-norm (messages are unit-trace in
  App. B; the global scale of the state is free);
* pseudo-inverses map zero to zero: 1/lambda for lambda = 0 (App. E) and
  mu^(-1/2) for message eigenvalues mu < eig_cut * mu_max (App. D);
* re-gauging (Sec. II.C steps i-iii) runs after every colour class by default;
  the paper re-gauges only "occasionally", when R (App. C) is too large: the
  "adaptive" policy reads that as R > res_max, tested after each class;
  its BP starts from the messages diag(lambda_ab)/sum(lambda_ab): with
  T = Gamma * prod(lambda^(1/2)) and local orthogonality these satisfy
  Eq. local_consistency exactly, whereas the printed Eq.
  reconstructed_messages carries lambda^(1/2) (kept as an option);
* BP (Alg. 1) updates edges in place in (colour, id) order; the distance is
  the trace norm (sum of |eigenvalues|) of the Hermitian difference; it stops
  when dist/|E| < tol or after max_sweeps sweeps.  tol <= 0 runs exactly
  max_sweeps sweeps (used for parity runs where the stop decision must not
  depend on rounding).  A Jacobi ("flooding") schedule is available too;
* readout uses the Vidal form: rho_a ~ sum Gamma Gamma* prod lambda^2, which
  equals Eq. partial_dens with the warm-start fixed-point messages; the bit is
  +1 iff rho_a[0,0] > 1/2 (Eq. rounding_rule).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .colouring import misra_gries

_LEG_KET = "abcdefgh"
_LEG_BRA = "ABCDEFGH"


@dataclass
class Options:
    chi: int = 4
    bp_tol: float = 1e-10
    bp_max_sweeps: int = 50
    svd_cut: float = 1e-12
    eig_cut: float = 1e-14
    regauge: str = "colour"        # "colour" | "step" | "never" | "adaptive"
    res_max: float = 1e-3          # "adaptive": re-gauge after a class only if R > res_max
    bp_schedule: str = "colour"    # "colour" (Gauss-Seidel, Alg. 1) | "flooding"
    warm_start: str = "lambda"     # "lambda" | "sqrt_lambda" (literal Eq. reconstructed_messages)


@dataclass
class State:
    """Vidal-gauge graph tensor network (Eq. vidal_gauge_tn)."""

    n: int
    edges: np.ndarray
    J: np.ndarray
    h: np.ndarray
    colour: np.ndarray
    inc: list            # inc[a] = incident edge ids of a, ascending (leg order)
    legpos: np.ndarray   # legpos[e] = (leg of e at u, leg of e at v)
    deg: np.ndarray
    gamma: list          # gamma[a]: complex [2, d_leg0, d_leg1, ...]
    lam: list            # lam[e]: float [d_e], non-negative, unit 2-norm
    opts: Options
    classes: list = field(default_factory=list)
    last_sweeps: list = field(default_factory=list)

    @property
    def n_edges(self):
        return int(self.edges.shape[0])

    def bond_dims(self):
        return np.array([lam.shape[0] for lam in self.lam])


# --------------------------------------------------------------------------
# construction and single-qubit gates
# --------------------------------------------------------------------------

def init_state(inst, opts: Options | None = None, colour=None) -> State:
    """|+>^N as a Vidal-gauge network with every bond of dimension 1
    (Sec. III.A: the initial product state has d_ab = 1)."""
    opts = opts or Options()
    n = inst.n
    edges = np.asarray(inst.edges, dtype=np.int64)
    m = edges.shape[0]
    inc = [[] for _ in range(n)]
    for e in range(m):
        inc[int(edges[e, 0])].append(e)
        inc[int(edges[e, 1])].append(e)
    for a in range(n):
        inc[a].sort()
    deg = np.array([len(x) for x in inc], dtype=np.int64)
    if (deg == 0).any():
        raise ValueError("isolated vertex: its field would never be applied")
    legpos = np.zeros((m, 2), dtype=np.int64)
    for e in range(m):
        u, v = int(edges[e, 0]), int(edges[e, 1])
        legpos[e, 0] = inc[u].index(e)
        legpos[e, 1] = inc[v].index(e)
    if colour is None:
        colour = misra_gries(n, edges)
    colour = np.asarray(colour, dtype=np.int64)
    ncol = int(colour.max()) + 1 if m else 0
    classes = [[e for e in range(m) if colour[e] == c] for c in range(ncol)]
    plus = np.array([1.0, 1.0], dtype=np.complex128) / np.sqrt(2.0)
    gamma = [plus.reshape((2,) + (1,) * int(deg[a])).copy() for a in range(n)]
    lam = [np.ones(1) for _ in range(m)]
    return State(n=n, edges=edges, J=np.asarray(inst.J, np.float64),
                 h=np.asarray(inst.h, np.float64), colour=colour, inc=inc,
                 legpos=legpos, deg=deg, gamma=gamma, lam=lam, opts=opts,
                 classes=classes)


def x_gate(theta: float) -> np.ndarray:
    """exp(-i theta X) = cos(theta) I - i sin(theta) X (App. F mixing layer)."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def apply_single_qubit(state: State, a: int, W: np.ndarray) -> None:
    """Gamma_a <- W . Gamma_a on the physical leg (Sec. II.D); the Vidal gauge
    is preserved because W is unitary."""
    state.gamma[a] = np.tensordot(W, state.gamma[a], axes=([1], [0]))


def x_layer(state: State, theta: float) -> None:
    W = x_gate(theta)
    for a in range(state.n):
        apply_single_qubit(state, a, W)


# --------------------------------------------------------------------------
# two-qubit gate: simple update (App. E) with truncation (Alg. 3)
# --------------------------------------------------------------------------

def zz_gate(theta: float, J: float, hu_D: float, hv_D: float) -> np.ndarray:
    """W[i_u, i_v, i_u', i_v'] of exp(-i theta (J Z_u Z_v + hu_D Z_u + hv_D Z_v)),
    a diagonal gate (App. F interaction layer)."""
    z = np.array([1.0, -1.0])
    W = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    for iu in range(2):
        for iv in range(2):
            W[iu, iv, iu, iv] = np.exp(-1j * theta * (J * z[iu] * z[iv]
                                                       + hu_D * z[iu] + hv_D * z[iv]))
    return W


def _scale_legs(G: np.ndarray, lams, skip: int | None, power: float = 1.0):
    """Multiply tensor G[i, j_0, j_1, ...] by prod_k lams[k][j_k]**power over legs k != skip."""
    out = G
    for k, lam in enumerate(lams):
        if k == skip:
            continue
        shape = [1] * G.ndim
        shape[1 + k] = lam.shape[0]
        out = out * (lam ** power).reshape(shape)
    return out


def _pinv_diag(lam: np.ndarray) -> np.ndarray:
    out = np.zeros_like(lam)
    nz = lam > 0
    out[nz] = 1.0 / lam[nz]
    return out


def _vertex_lams(state: State, a: int):
    return [state.lam[e] for e in state.inc[a]]


def simple_update(state: State, e: int, theta: float):
    """Apply the interaction gate of edge e (App. E).

    Theta = W . Gamma_u lambda_e Gamma_v . prod(outer lambdas); SVD over the
    split (i_u, outer legs of u) | (i_v, outer legs of v); keep at most chi
    values (Alg. 3); Gamma_u <- U / outer lambdas, Gamma_v <- V^dagger / outer
    lambdas, lambda_e <- kept singular values (unit 2-norm).

    Returns (f, eps): the gate-fidelity estimate (Eq. gate_fidelity, computed
    on the normalised spectrum before truncation) and the edge truncation
    error eps_ab^chi (Sec. II.C).
    """
    opts = state.opts
    u, v = int(state.edges[e, 0]), int(state.edges[e, 1])
    pu, pv = int(state.legpos[e, 0]), int(state.legpos[e, 1])
    W = zz_gate(theta, state.J[e], state.h[u] / state.deg[u], state.h[v] / state.deg[v])
    lam_u = _vertex_lams(state, u)
    lam_v = _vertex_lams(state, v)
    A = _scale_legs(state.gamma[u], lam_u, skip=pu)
    B = _scale_legs(state.gamma[v], lam_v, skip=pv)
    A = np.moveaxis(A, 1 + pu, -1)          # [i_u, outer_u..., j]
    B = np.moveaxis(B, 1 + pv, -1)          # [i_v, outer_v..., j]
    outer_u = A.shape[1:-1]
    outer_v = B.shape[1:-1]
    Ru = int(np.prod(outer_u, dtype=np.int64))
    Rv = int(np.prod(outer_v, dtype=np.int64))
    lam_e = state.lam[e]
    # Theta0[i_u', (outer_u), i_v', (outer_v)] = sum_j A[..., j] lambda_e[j] B[..., j]
    Th0 = (A.reshape(2 * Ru, -1) * lam_e[None, :]) @ B.reshape(2 * Rv, -1).T
    Th0 = Th0.reshape(2, Ru, 2, Rv)
    Th = np.einsum("abcd,cxdy->axby", W, Th0).reshape(2 * Ru, 2 * Rv)
    U, s, Vh = np.linalg.svd(Th, full_matrices=False)
    r = int(min(opts.chi, np.count_nonzero(s > opts.svd_cut * s[0])))
    tot = float(np.sum(s * s))
    kept = float(np.sum(s[:r] ** 2))
    f = (kept / tot) ** 2
    eps = float(np.sqrt(np.sum(s[r:] ** 2) / tot))
    lam_new = s[:r] / np.linalg.norm(s[:r])
    Gu = U[:, :r].reshape((2,) + outer_u + (r,))
    Gv = Vh[:r, :].T.reshape((2,) + outer_v + (r,))
    Gu = np.moveaxis(Gu, -1, 1 + pu)
    Gv = np.moveaxis(Gv, -1, 1 + pv)
    inv_u = [_pinv_diag(x) for x in lam_u]
    inv_v = [_pinv_diag(x) for x in lam_v]
    state.gamma[u] = _scale_legs(Gu, inv_u, skip=pu)
    state.gamma[v] = _scale_legs(Gv, inv_v, skip=pv)
    state.lam[e] = lam_new
    return f, eps


# --------------------------------------------------------------------------
# re-gauging: symmetric gauge, BP (Alg. 1), Vidal gauge from messages (Alg. 2)
# --------------------------------------------------------------------------

def symmetric_gauge(state: State):
    """T_a = Gamma_a prod_b lambda_ba^(1/2) (Eq. symmetric_gauge)."""
    return [_scale_legs(state.gamma[a], _vertex_lams(state, a), skip=None, power=0.5)
            for a in range(state.n)]


def warm_messages(state: State):
    """Warm-start messages from lambda (Sec. II.C).  msgs[e] = [m_{u->v}, m_{v->u}]."""
    msgs = []
    for e in range(state.n_edges):
        lam = state.lam[e]
        w = lam if state.opts.warm_start == "lambda" else np.sqrt(lam)
        m = np.diag(w / w.sum()).astype(np.complex128)
        msgs.append([m, m.copy()])
    return msgs


def random_messages(state: State, entries):
    """Alg. 1's random initialisation m = A A^dagger / tr(A A^dagger) from given
    entries: entries[e][dir] is a complex d_e x d_e matrix A."""
    msgs = []
    for e in range(state.n_edges):
        pair = []
        for d in range(2):
            A = np.asarray(entries[e][d], dtype=np.complex128)
            M = A @ A.conj().T
            pair.append(M / np.trace(M).real)
        msgs.append(pair)
    return msgs


def incoming(state: State, msgs, a: int, e: int):
    """Message arriving at vertex a along edge e (from the other endpoint)."""
    u = int(state.edges[e, 0])
    return msgs[e][1] if a == u else msgs[e][0]


def message_update(T_a: np.ndarray, out_leg: int, incoming_by_leg) -> np.ndarray:
    """Eq. local_consistency: m_{a->b}[j, j'] = sum T_a[i, j, ...] T_a*[i, j', ...]
    prod_{c != b} m_{c->a}[k_c, k'_c], with j the leg toward b.

    Evaluated as: contract each incoming message into T_a's ket legs in leg
    order, then contract the result with T_a* over i and the primed legs."""
    deg = T_a.ndim - 1
    Tm = np.moveaxis(T_a, 1 + out_leg, 1)          # [i, j, other legs in order]
    others = [k for k in range(deg) if k != out_leg]
    K = Tm
    for k in others:
        # the next unprimed leg is always axis 2; its primed copy goes last
        K = np.tensordot(K, incoming_by_leg[k], axes=([2], [0]))
    ax = [0] + list(range(2, deg + 1))
    return np.tensordot(K, Tm.conj(), axes=(ax, ax))


def trace_norm(D: np.ndarray) -> float:
    """||D||_1 = sum |eigenvalues| for Hermitian D."""
    return float(np.sum(np.abs(np.linalg.eigvalsh(D))))


def _new_messages_for_edge(state: State, T, msgs, e: int):
    out = []
    for side in range(2):
        a = int(state.edges[e, side])
        p = int(state.legpos[e, side])
        inc_by_leg = {}
        for k, e2 in enumerate(state.inc[a]):
            if k != p:
                inc_by_leg[k] = incoming(state, msgs, a, e2)
        m = message_update(T[a], p, inc_by_leg)
        # unit trace (App. B) by the complex trace: dividing by its real part
        # would leave a complex scale on m that the multilinear update of
        # Alg. 1 compounds from sweep to sweep
        out.append(m / np.trace(m))
    return out


def bp_order(state: State):
    """Edges sorted by (colour, id): the in-place update order of Alg. 1."""
    return sorted(range(state.n_edges), key=lambda e: (int(state.colour[e]), e))


def belief_propagation(state: State, T, msgs, tol: float, max_sweeps: int,
                       schedule: str = "colour"):
    """Alg. 1 on tensors T starting from `msgs` (updated in place).
    Returns (sweeps_done, dist / |E| of the last sweep)."""
    m_edges = state.n_edges
    order = bp_order(state)
    dist_avg = 0.0
    sweeps = 0
    for _ in range(max_sweeps):
        sweeps += 1
        dist = 0.0
        if schedule == "colour":
            for e in order:
                new = _new_messages_for_edge(state, T, msgs, e)
                for d in range(2):
                    dist += trace_norm(new[d] - msgs[e][d])
                    msgs[e][d] = new[d]
        elif schedule == "flooding":
            news = [_new_messages_for_edge(state, T, msgs, e) for e in range(m_edges)]
            for e in range(m_edges):
                for d in range(2):
                    dist += trace_norm(news[e][d] - msgs[e][d])
                    msgs[e][d] = news[e][d]
        else:
            raise ValueError(schedule)
        dist_avg = dist / m_edges
        if dist_avg < tol:
            break
    return sweeps, dist_avg


def sqrt_and_pinv_sqrt(m: np.ndarray, eig_cut: float):
    """m^(1/2) and the pseudo-inverse m^(-1/2) of a Hermitian PSD message."""
    mu, W = np.linalg.eigh(m)
    mu_max = float(np.max(mu))
    keep = mu > eig_cut * mu_max
    sq = np.where(keep, np.sqrt(np.where(keep, mu, 1.0)), 0.0)
    isq = np.where(keep, 1.0 / np.where(keep, sq, 1.0), 0.0)
    S = (W * sq[None, :]) @ W.conj().T
    Sinv = (W * isq[None, :]) @ W.conj().T
    return S, Sinv


def _apply_leg(G: np.ndarray, leg: int, X: np.ndarray) -> np.ndarray:
    """G'[..., q@leg, ...] = sum_j G[..., j@leg, ...] X[j, q]."""
    out = np.tensordot(G, X, axes=([1 + leg], [0]))   # leg moved to the end
    return np.moveaxis(out, -1, 1 + leg)


def vidal_from_messages(state: State, T, msgs) -> None:
    """Alg. 2: Gamma_a <- T_a, then for every edge {a, b}: SVD of
    C[k, l] = sum_j m_{a->b}^(1/2)[j, k] m_{b->a}^(1/2)[j, l] and
    Gamma_a <- Gamma_a x (m_{a->b}^(-1/2))^T U,  Gamma_b <- Gamma_b x (m_{b->a}^(-1/2))^T V*,
    lambda_ab <- singular values (kept above svd_cut * sigma_0, unit 2-norm)."""
    opts = state.opts
    gamma = [t.copy() for t in T]
    lam = list(state.lam)
    for e in range(state.n_edges):
        u, v = int(state.edges[e, 0]), int(state.edges[e, 1])
        pu, pv = int(state.legpos[e, 0]), int(state.legpos[e, 1])
        S_uv, Si_uv = sqrt_and_pinv_sqrt(msgs[e][0], opts.eig_cut)
        S_vu, Si_vu = sqrt_and_pinv_sqrt(msgs[e][1], opts.eig_cut)
        C = S_uv.T @ S_vu
        U, s, Vh = np.linalg.svd(C)
        r = int(np.count_nonzero(s > opts.svd_cut * s[0]))
        lam[e] = s[:r] / np.linalg.norm(s[:r])
        X_u = Si_uv.T @ U[:, :r]
        X_v = Si_vu.T @ Vh[:r, :].T
        gamma[u] = _apply_leg(gamma[u], pu, X_u)
        gamma[v] = _apply_leg(gamma[v], pv, X_v)
    state.gamma = gamma
    state.lam = lam


def regauge(state: State):
    """Sec. II.C re-gauging: (i) symmetric gauge, (ii) BP from warm messages,
    (iii) Vidal gauge from the messages.  Returns (sweeps, dist/|E|)."""
    opts = state.opts
    T = symmetric_gauge(state)
    msgs = warm_messages(state)
    sweeps, dist = belief_propagation(state, T, msgs, opts.bp_tol, opts.bp_max_sweeps,
                                      opts.bp_schedule)
    vidal_from_messages(state, T, msgs)
    return sweeps, dist


def truncate_edge(state: State, e: int, chi: int) -> float:
    """Alg. 3: keep the chi largest Schmidt values of edge e (lambda is sorted
    descending) and the matching slices of Gamma_u, Gamma_v.  No
    renormalisation.  Returns eps_ab^chi = sqrt(sum of dropped lambda^2)."""
    lam = state.lam[e]
    eps = float(np.sqrt(np.sum(lam[chi:] ** 2)))
    u, v = int(state.edges[e, 0]), int(state.edges[e, 1])
    pu, pv = int(state.legpos[e, 0]), int(state.legpos[e, 1])
    state.lam[e] = lam[:chi].copy()
    state.gamma[u] = np.take(state.gamma[u], np.arange(min(chi, lam.size)), axis=1 + pu)
    state.gamma[v] = np.take(state.gamma[v], np.arange(min(chi, lam.size)), axis=1 + pv)
    return eps


def vidal_residual(state: State) -> float:
    """R of App. C: (1/2|E|) sum over directions a->b of the trace norm of
    delta - M_{a->b}, M = sum Gamma_a Gamma_a* prod_{c != b} lambda_ca^2.

    Reading: Alg. 2 fixes each Gamma_a only up to a positive scale (messages
    are unit-trace, lambda unit-norm), and the state's norm is free, so M is
    compared with the identity after dividing by its mean eigenvalue
    tr(M)/d_ab.  A Gram that is a multiple of the identity in one direction
    has the same multiple in every direction of that vertex, so this loses
    no information about local orthogonality."""
    tot = 0.0
    for a in range(state.n):
        lams = _vertex_lams(state, a)
        for p in range(len(state.inc[a])):
            G = state.gamma[a]
            Gw = _scale_legs(G, lams, skip=p, power=2.0)
            A = np.moveaxis(G, 1 + p, -1).reshape(-1, G.shape[1 + p])
            B = np.moveaxis(Gw, 1 + p, -1).reshape(-1, G.shape[1 + p])
            M = A.T @ B.conj()          # [j, j'] = sum Gamma[.., j] Gamma*[.., j'] lambda^2
            M = 0.5 * (M + M.conj().T)
            M = M * (M.shape[0] / np.trace(M).real)
            tot += trace_norm(np.eye(M.shape[0]) - M)
    return tot / (2.0 * state.n_edges)


# --------------------------------------------------------------------------
# Trotter step, readout, objective
# --------------------------------------------------------------------------

@dataclass
class StepStats:
    sweeps: list = field(default_factory=list)    # BP sweeps per re-gauge
    dists: list = field(default_factory=list)     # final dist/|E| per re-gauge
    log_fidelity: float = 0.0                      # sum log f over the step's gates
    max_eps: float = 0.0
    residuals: list = field(default_factory=list)  # "adaptive": R after each class


def trotter_step(state: State, theta_z: float, theta_x: float) -> StepStats:
    """One first-order Trotter step: U_Z(theta_z) class by class (each class
    followed by re-gauging under the default policy, or under "adaptive" only
    where R exceeds res_max), then U_X(theta_x)."""
    st = StepStats()
    pol = state.opts.regauge
    for cls in state.classes:
        for e in cls:
            f, eps = simple_update(state, e, theta_z)
            st.log_fidelity += float(np.log(f))
            st.max_eps = max(st.max_eps, eps)
        if pol == "colour" and cls:
            s, d = regauge(state)
            st.sweeps.append(s)
            st.dists.append(d)
        elif pol == "adaptive" and cls:
            # occasional re-gauging (Sec. II.C): only once the state has
            # drifted from the Vidal gauge by more than res_max in R (App. C)
            r = vidal_residual(state)
            st.residuals.append(r)
            if r > state.opts.res_max:
                s, d = regauge(state)
                st.sweeps.append(s)
                st.dists.append(d)
    if pol == "step":
        s, d = regauge(state)
        st.sweeps.append(s)
        st.dists.append(d)
    x_layer(state, theta_x)
    state.last_sweeps = st.sweeps
    return st


def rho_vidal(state: State) -> np.ndarray:
    """rho_a[i, i'] ~ sum_J Gamma_a[i, J] Gamma_a*[i', J] prod_legs lambda^2, unit trace."""
    out = np.zeros((state.n, 2, 2), dtype=np.complex128)
    for a in range(state.n):
        G = state.gamma[a]
        Gw = _scale_legs(G, _vertex_lams(state, a), skip=None, power=2.0)
        r = G.reshape(2, -1) @ Gw.reshape(2, -1).conj().T
        out[a] = r / np.trace(r).real
    return out


def rho_messages(state: State, T, msgs) -> np.ndarray:
    """Eq. partial_dens with the environment of Eq. bp_approx, unit trace."""
    out = np.zeros((state.n, 2, 2), dtype=np.complex128)
    for a in range(state.n):
        Ta = T[a]
        deg = Ta.ndim - 1
        spec_k = "i" + _LEG_KET[:deg]
        spec_b = "j" + _LEG_BRA[:deg]
        ops = [Ta, Ta.conj()]
        subs = []
        for k, e in enumerate(state.inc[a]):
            ops.append(incoming(state, msgs, a, e))
            subs.append(_LEG_KET[k] + _LEG_BRA[k])
        r = np.einsum(spec_k + "," + spec_b + "," + ",".join(subs) + "->ij", *ops,
                      optimize=True)
        out[a] = r / np.trace(r).real
    return out


def z_expectations(rho: np.ndarray) -> np.ndarray:
    return (rho[:, 0, 0] - rho[:, 1, 1]).real


def rounding(rho: np.ndarray) -> np.ndarray:
    """Eq. rounding_rule: x_a = +1 if rho_a[0,0] > 1/2 else -1."""
    return np.where(rho[:, 0, 0].real > 0.5, 1, -1).astype(np.int8)


def objective(edges: np.ndarray, J: np.ndarray, h: np.ndarray, x: np.ndarray) -> float:
    """Eq. objective_function E(x) = sum_e J_e x_u x_v + sum_a h_a x_a."""
    x = np.asarray(x, dtype=np.float64)
    return float(np.sum(J * x[edges[:, 0]] * x[edges[:, 1]]) + np.sum(h * x))


def readout(state: State):
    rho = rho_vidal(state)
    x = rounding(rho)
    return z_expectations(rho), rho, x, objective(state.edges, state.J, state.h, x)


def run_angles(inst, theta_z, theta_x, theta_x0: float = 0.0, opts: Options | None = None, colour=None):
    """A product formula given as angles (inputs): U_X(theta_x0) on |+>^N,
    then Trotter steps (theta_z[k], theta_x[k]).  With theta_x0 = 0 and the
    angles of App. F this is the first-order anneal; the symmetric
    second-order formula (Sec. VI names higher-order formulas) is the same
    sequence with midpoint angles and merged half mixing layers."""
    state = init_state(inst, opts, colour)
    if theta_x0 != 0.0:
        x_layer(state, theta_x0)
    stats = [trotter_step(state, tz, tx) for tz, tx in zip(theta_z, theta_x)]
    return state, stats


def anneal(inst, T: float, dt: float, opts: Options | None = None, colour=None,
           record_z: bool = False, checkpoints=(), on_checkpoint=None):
    """GTQA (Sec. III.A): start from |+>^N, apply the Trotter circuit of App. F
    with s(t) = 1 - t/T, read out.  Returns the final state and a dict with
    per-step <Z> (if requested), checkpoint readouts and per-step statistics.
    `on_checkpoint(k, out, state)`, if given, is called after each
    checkpoint's readout (long runs save their progress there); it must not
    modify the state."""
    state = init_state(inst, opts, colour)
    K = int(round(T / dt))
    out = {"z": [], "checkpoints": {}, "stats": []}
    cps = set(checkpoints)
    for k in range(1, K + 1):
        # s_k = s(k dt) = 1 - k/K: theta_z = dt (1 - s_k), theta_x = dt s_k
        theta_z = dt * k / K
        theta_x = dt * (K - k) / K
        out["stats"].append(trotter_step(state, theta_z, theta_x))
        if record_z or k in cps:
            z, rho, x, E = readout(state)
            if record_z:
                out["z"].append(z)
            if k in cps:
                out["checkpoints"][k] = {"z": z, "x": x, "E": E}
                if on_checkpoint is not None:
                    on_checkpoint(k, out, state)
    return state, out
