"""The C ABI's less travelled calls on the GPU, against the oracle.

* gtqa_bond_svd: the simple update's bond SVD (Alg. 3 keeps the chi largest
  Schmidt values) on adversarial cores whose discarded columns hide a larger
  singular value, on graded random cores, and on rank-deficient ones; the
  kept values must equal LAPACK's chi largest (Eckart-Young).
* gtqa_bp_converge with Alg. 1's random start (App. B): exact rho on a tree
  (BP is exact on trees from any start, Sec. II.B), and the oracle's messages
  and distance after a fixed number of sweeps from the same random messages
  on a loopy graph.
* GTQA_WARN_BP_MAXITER when the sweep cap K of Alg. 1 is reached first.
* gtqa_set_network / gtqa_get_network: round trip, and one Trotter step from
  a network the oracle produced, compared with the oracle's step.
"""

import numpy as np
import pytest

from oracle import gtqa as O
from synthetic import (random_message_entries, random_regular_instance, random_tree_instance,
                       schedule_angles)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    from paper_2409_12240_amd import gtqa
    return gtqa.TorchDevice()


def _state(inst, dev, **kw):
    from paper_2409_12240_amd import gtqa
    return gtqa.TrotterState(inst, device=dev, **kw)


def _adversarial(rng, hidden):
    Q, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
    M = np.zeros((8, 8), dtype=np.complex128)
    M[:, :4] = Q[:, :4]
    M[:, 4:] = hidden * Q[:, 4:5]
    return M


def test_bond_svd_keeps_the_largest_values_chi4():
    from paper_2409_12240_amd import gtqa
    rng = np.random.default_rng(21)
    cores = []
    for hidden in np.linspace(0.5, 0.99, 24):          # hidden value 2*hidden > 1 behind norms < 1
        cores.append(_adversarial(rng, hidden))
    for _ in range(24):                                  # ... also mixed with noise and permuted
        M = _adversarial(rng, rng.uniform(0.5, 0.99))
        M[:, 4:] += 0.05 * (rng.normal(size=(8, 4)) + 1j * rng.normal(size=(8, 4)))
        cores.append(M[:, rng.permutation(8)])
    for _ in range(200):                                 # graded spectra
        U, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
        V, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
        sig = rng.uniform(0.2, 0.9) ** np.arange(8) * rng.uniform(0.8, 1.2, 8)
        cores.append((U * sig) @ V.conj().T)
    a = rng.normal(size=(8, 2)) + 1j * rng.normal(size=(8, 2))   # rank 2
    b = rng.normal(size=(8, 2)) + 1j * rng.normal(size=(8, 2))
    cores.append(a @ b.conj().T)
    cores = np.stack(cores)
    sig, sweeps = gtqa.bond_svd(4, cores)
    exact = np.linalg.svd(cores, compute_uv=False)
    print(f"{len(cores)} cores: sweeps mean {sweeps.mean():.2f}, max {sweeps.max()}", flush=True)
    assert sweeps.max() <= 40
    np.testing.assert_allclose(sig[:, :4], exact[:, :4], rtol=1e-12, atol=1e-13)
    # the total norm of the core is kept exactly (the discarded part feeds eps and f)
    np.testing.assert_allclose(np.sum(sig ** 2, axis=1), np.sum(exact ** 2, axis=1), rtol=1e-13)


def test_bond_svd_chi8_full_spectrum():
    from paper_2409_12240_amd import gtqa
    rng = np.random.default_rng(22)
    cores = []
    for _ in range(64):
        U, _ = np.linalg.qr(rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16)))
        V, _ = np.linalg.qr(rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16)))
        sig = rng.uniform(0.3, 0.95) ** np.arange(16)
        cores.append((U * sig) @ V.conj().T)
    cores = np.stack(cores)
    sig, sweeps = gtqa.bond_svd(8, cores)
    exact = np.linalg.svd(cores, compute_uv=False)
    np.testing.assert_allclose(sig, exact, rtol=1e-11, atol=1e-13)


def test_bond_svd_rejects_bad_input():
    from paper_2409_12240_amd import gtqa
    c = np.zeros((1, 8, 8), dtype=np.complex128)
    c[0, 0, 0] = np.nan
    with pytest.raises(gtqa.GtqaError) as ei:
        gtqa.bond_svd(4, c)
    assert ei.value.code == gtqa.GTQA_ERR_NUMERIC
    with pytest.raises(gtqa.GtqaError) as ei:
        gtqa.bond_svd(5, np.zeros((1, 10, 10)))
    assert ei.value.code == gtqa.GTQA_ERR_UNSUPPORTED


def test_bp_random_start_on_a_tree_is_exact(dev):
    # BP is exact on trees whatever its start (Sec. II.B): from Alg. 1's
    # random messages it must reach the state vector's single-qubit rho
    from oracle import exact as X
    inst = random_tree_instance(3, 12)
    T, dt = 2.0, 0.25
    tz, tx = schedule_angles(T, dt)
    _, rex = X.anneal_statevector(inst, T, dt)
    st = _state(inst, dev, chi=8, bp_tol=0.0, bp_max_sweeps=12)
    for k in range(tz.size):
        st.step(tz[k], tx[k])
    for seed in (1, 2**63 + 5):
        rc, sw, dist = st.bp_converge(1e-14, 500, random_seed=seed)
        assert rc == 0 and sw < 500
        r = st.readout(from_messages=True)
        np.testing.assert_allclose(r["rho"], rex[-1], atol=1e-10)
    st.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-4)])
def test_bp_random_start_matches_oracle_on_a_loopy_graph(dev, precision, tol):
    # A random start is not gauge invariant: the library's Jacobi SVD and
    # LAPACK leave different phases on the singular vectors, so after
    # independent evolutions the two networks differ by phases on every bond
    # and the same random matrices are different messages.  The oracle's
    # network is therefore loaded into the library first.
    inst = random_regular_instance(6, 16)
    tz, tx = schedule_angles(10.0, 0.1)
    ost = O.init_state(inst, O.Options(chi=4, bp_tol=0.0, bp_max_sweeps=6))
    for k in range(15):
        O.trotter_step(ost, tz[k], tx[k])
    st = _state(inst, dev, chi=4, precision=precision, bp_tol=0.0, bp_max_sweeps=6)
    st.set_network(*_oracle_network(ost, 4))
    seed = 0x5EED
    for sweeps in (1, 9):
        rc, sw, dist = st.bp_converge(0.0, sweeps, random_seed=seed)
        assert rc == 0 and sw == sweeps
        T = O.symmetric_gauge(ost)
        msgs = O.random_messages(ost, random_message_entries(seed, ost.bond_dims(), 4))
        _, odist = O.belief_propagation(ost, T, msgs, 0.0, sweeps)
        r = st.readout(from_messages=True)
        rho_o = O.rho_messages(ost, T, msgs)
        worst = float(np.max(np.abs(r["rho"] - rho_o)))
        print(f"{precision} random start, {sweeps} sweeps: max |d rho| {worst:.2e}, "
              f"dist {dist:.6e} vs {odist:.6e}", flush=True)
        assert worst < tol
        assert abs(dist - odist) < tol * max(1.0, odist)
    st.close()


def test_bp_random_start_reaches_the_warm_fixed_point(dev):
    # Alg. 1 from random messages and from the warm start meet at the same
    # fixed point on this loopy graph (the paper accepts any fixed point;
    # here there is one), well inside the stop tolerance
    inst = random_regular_instance(7, 16)
    tz, tx = schedule_angles(10.0, 0.1)
    st = _state(inst, dev, chi=4, bp_tol=1e-12, bp_max_sweeps=100)
    for k in range(20):
        st.step(tz[k], tx[k])
    st.bp_converge(1e-13, 400)
    warm = st.readout(from_messages=True)["rho"]
    rc, sw, _ = st.bp_converge(1e-13, 400, random_seed=99)
    assert rc == 0 and sw > 1
    rnd = st.readout(from_messages=True)["rho"]
    assert float(np.max(np.abs(warm - rnd))) < 1e-9
    st.close()


def test_bp_sweep_cap_warns(dev):
    # K of Alg. 1 reached before the stop test: a warning, results written
    from paper_2409_12240_amd import gtqa
    inst = random_regular_instance(8, 16)
    tz, tx = schedule_angles(10.0, 0.1)
    st = _state(inst, dev, chi=4, bp_tol=1e-30, bp_max_sweeps=1)
    rcs = [st.step(tz[k], tx[k]) for k in range(5)]
    assert rcs[-1] == gtqa.GTQA_WARN_BP_MAXITER
    rc, sw, dist = st.bp_converge(1e-30, 2)
    assert rc == gtqa.GTQA_WARN_BP_MAXITER and sw == 2 and dist > 1e-30
    rc, sw, _ = st.bp_converge(1.0, 2)
    assert rc == gtqa.GTQA_OK and sw == 1
    assert np.isfinite(st.readout()["z"]).all()
    st.close()


def _oracle_network(ost, chi):
    g = np.zeros((ost.n, 2, chi, chi, chi), dtype=np.complex128)
    for a in range(ost.n):
        G = ost.gamma[a]
        G = G.reshape(G.shape + (1,) * (4 - G.ndim))
        g[a][tuple(slice(0, d) for d in G.shape)] = G
    lam = np.zeros((ost.n_edges, chi))
    for e in range(ost.n_edges):
        lam[e, :ost.lam[e].size] = ost.lam[e]
    return g, lam


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_network_round_trip(dev, precision):
    inst = random_regular_instance(9, 16)
    tz, tx = schedule_angles(10.0, 0.1)
    ost = O.init_state(inst, O.Options(chi=4))
    for k in range(25):
        O.trotter_step(ost, tz[k], tx[k])
    g, lam = _oracle_network(ost, 4)
    st = _state(inst, dev, chi=4, precision=precision)
    st.set_network(g, lam)
    g2, lam2 = st.get_network()
    assert np.array_equal(lam2, lam)
    if precision == "fp64":
        assert np.array_equal(g2, g)
    else:
        np.testing.assert_allclose(g2, g, atol=1e-7 * np.abs(g).max())
    # the readout of the loaded network is the oracle's
    zo = O.readout(ost)[0]
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert float(np.max(np.abs(st.readout()["z"] - zo))) < tol
    from paper_2409_12240_amd import gtqa
    bad = lam.copy()
    bad[0, :] = bad[0, ::-1]
    with pytest.raises(gtqa.GtqaError):
        st.set_network(g, bad)
    st.close()


@pytest.mark.parametrize("chi", [4, 8])
def test_one_step_from_an_oracle_network(dev, chi):
    # mid-anneal, where truncation acts and BP needs several sweeps: the
    # oracle's network after k steps goes into the library, both sides take
    # step k + 1 with the tolerance stop of the anneal (1e-10, 50 sweeps)
    inst = random_regular_instance(10, 24)
    tz, tx = schedule_angles(10.0, 0.1)
    ost = O.init_state(inst, O.Options(chi=chi))
    for k in range(50):
        O.trotter_step(ost, tz[k], tx[k])
    g, lam = _oracle_network(ost, chi)
    st = _state(inst, dev, chi=chi, bp_tol=1e-10, bp_max_sweeps=50)
    st.set_network(g, lam)
    _, gs = st.step(tz[50], tx[50], stats=True)
    os_ = O.trotter_step(ost, tz[50], tx[50])
    zo = O.readout(ost)[0]
    dz = float(np.max(np.abs(st.readout()["z"] - zo)))
    print(f"chi={chi}: sweeps {gs['bp_sweeps']} vs {os_.sweeps}, max |dz| {dz:.2e}", flush=True)
    assert list(gs["bp_sweeps"]) == list(os_.sweeps)
    assert max(os_.sweeps) > 1
    assert dz < 1e-10
    st.close()
