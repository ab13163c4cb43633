"""The kept-column Jacobi rule of the chi <= 4 simple update, on the CPU.

The library's bond SVD (Alg. 3 keeps the chi largest Schmidt values) runs a
one-sided Jacobi iteration that, to save sweeps, rotates only column pairs
that touch one of the chi largest columns (ranked by norm at the start of
each sweep).  At convergence those columns are exact singular triplets, but
nothing in the rule itself makes them the chi LARGEST: discarded columns are
never rotated against each other, so correlated discarded columns can hide a
larger singular value.  The library therefore checks, once the kept columns
have converged, that the discarded columns' total squared norm (an upper
bound on the square of their largest singular value, since they are
orthogonal to the kept ones) lies below the smallest kept squared norm, or
below the relative cutoff under which values are dropped anyway; otherwise it
continues with rotations on every pair, i.e. the plain one-sided Jacobi SVD.
The restricted rule also need not converge at all when weight keeps moving
between the kept and the discarded columns, so after a fixed number of
restricted sweeps the iteration switches to every pair as well.

`model_team_svd` below is a NumPy model of the device routine's decisions
(pairing c with c ^ r in round r, kept set by rank, stop test, guard); the
rotations use exact arithmetic instead of the hardware approximations, which
only change how fast gamma vanishes.  Tests: an adversarial core on which the
rule without the guard keeps the wrong values, and random graded cores, each
compared with LAPACK's singular values (the Eckart-Young choice).
"""

import numpy as np
import pytest


def _ranks(own):
    n = own.size
    return np.array([sum(1 for c in range(n) if own[c] > own[i] or (own[c] == own[i] and c < i))
                     for i in range(n)])


def model_team_svd(M, keep, guard=True, tol=1e-15, max_sweeps=40, cut=1e-12, keep_sweeps=16):
    """Columns of M rotated as the device team does; returns (columns, sweeps, went_full)."""
    M = np.array(M, dtype=np.complex128)
    N = M.shape[1]
    eps2 = tol / (20.0 * max(N - 2, 1))
    full = keep >= N
    for sweep in range(max_sweeps):
        if guard and not full and sweep >= keep_sweeps:
            full = True            # the kept set has not settled: plain Jacobi
        own = np.sum(np.abs(M) ** 2, axis=0)
        kept = np.ones(N, bool) if full else _ranks(own) < keep
        rotated = big = False
        for r in range(1, N):
            pairs = [(p, p ^ r) for p in range(N) if (p ^ r) > p]
            for p, q in pairs:                 # disjoint pairs: any order
                g = np.vdot(M[:, p], M[:, q])
                g2 = abs(g) ** 2
                rot = g2 > 0 and g2 > tol * tol * own[p] * own[q] and (kept[p] or kept[q])
                if not rot:
                    continue
                rotated = True
                d = 0.5 * (own[q] - own[p])
                tau = np.sign(d if d != 0 else 1.0) / (abs(d) + np.sqrt(d * d + g2))
                c = 1.0 / np.sqrt(1.0 + tau * tau * g2)
                s = c * tau * g
                mp, mq = M[:, p].copy(), M[:, q].copy()
                M[:, p] = c * mp - np.conj(s) * mq
                M[:, q] = s * mp + c * mq
                tg = tau * g2
                own[p] -= tg
                own[q] += tg
                if g2 > eps2 * own[p] * own[q] or tau * tg > eps2:
                    big = True
        st = 0 if not rotated else (2 if big else 1)
        if not full and st == 1:
            now = _ranks(own) < keep
            st = 2 if (now != kept).any() else 1
        if st < 2:
            if not full and guard:
                own = np.sum(np.abs(M) ** 2, axis=0)
                rk = _ranks(own)
                dsum = float(np.sum(own[rk >= keep]))
                kmin = float(np.min(own[rk < keep]))
                if not (dsum < kmin or dsum <= cut * cut * float(np.max(own))):
                    full = True
                    continue
            return M, sweep + 1, full
    return M, max_sweeps + 1, full


def kept_sigma(M, keep, **kw):
    cols, sweeps, full = model_team_svd(M, keep, **kw)
    s = np.sort(np.linalg.norm(cols, axis=0))[::-1]
    return s[:keep], sweeps, full


def adversarial_core(rng, n=8, keep=4, hidden=0.9):
    """Columns 0..keep-1 orthonormal; the other columns all equal to one vector
    of norm `hidden` orthogonal to them.  The discarded block has singular
    value hidden * sqrt(n - keep) > 1, hidden behind column norms below 1."""
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    M = np.zeros((n, n), dtype=np.complex128)
    M[:, :keep] = Q[:, :keep]
    for c in range(keep, n):
        M[:, c] = hidden * Q[:, keep]
    return M


def test_rule_without_guard_keeps_the_wrong_values():
    M = adversarial_core(np.random.default_rng(1))
    exact = np.linalg.svd(M, compute_uv=False)[:4]
    s, _, _ = kept_sigma(M, 4, guard=False)
    assert exact[0] == pytest.approx(0.9 * 2.0, rel=1e-12)
    np.testing.assert_allclose(s, 1.0, rtol=1e-12)       # the hidden 1.8 is missed
    assert abs(s[0] - exact[0]) > 0.5


@pytest.mark.parametrize("seed", range(5))
def test_guard_recovers_the_largest_values_on_adversarial_cores(seed):
    rng = np.random.default_rng(seed)
    for hidden in (0.51, 0.6, 0.9, 0.99):
        M = adversarial_core(rng, hidden=hidden)
        exact = np.linalg.svd(M, compute_uv=False)[:4]
        s, _, full = kept_sigma(M, 4)
        assert full
        np.testing.assert_allclose(s, exact, rtol=1e-12, atol=1e-14)


def test_guard_on_correlated_discards_mixed_with_the_kept_span():
    # discarded columns correlated among themselves and partly inside the
    # kept span: rotations happen before the hidden value shows
    rng = np.random.default_rng(7)
    for _ in range(200):
        M = adversarial_core(rng, hidden=rng.uniform(0.5, 0.99))
        M[:, 4:] += 0.05 * (rng.normal(size=(8, 4)) + 1j * rng.normal(size=(8, 4)))
        M = M[:, rng.permutation(8)]
        exact = np.linalg.svd(M, compute_uv=False)[:4]
        s, _, _ = kept_sigma(M, 4)
        np.testing.assert_allclose(s, exact, rtol=1e-11, atol=1e-13)


def test_random_graded_cores_keep_the_largest_values():
    # spectra decaying by 0.2 .. 0.9 per index: flat ones trip the guard (the
    # cores of an anneal almost never do: their tails are far below sigma_chi)
    rng = np.random.default_rng(11)
    n_full = 0
    for t in range(400):
        decay = rng.uniform(0.2, 0.9)
        U, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
        V, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
        sig = decay ** np.arange(8) * rng.uniform(0.8, 1.2, 8)
        M = (U * sig) @ V.conj().T
        exact = np.linalg.svd(M, compute_uv=False)[:4]
        s, _, full = kept_sigma(M, 4)
        n_full += full
        np.testing.assert_allclose(s, exact, rtol=1e-11, atol=1e-14)
    print(f"{n_full} of 400 graded cores continued with every pair")


def test_zero_tail_passes_the_guard_by_the_cutoff():
    # rank-2 core (the first steps of an anneal): kept and discarded tails are
    # both at rounding level; the guard accepts through the relative cutoff
    rng = np.random.default_rng(3)
    a = rng.normal(size=(8, 2)) + 1j * rng.normal(size=(8, 2))
    b = rng.normal(size=(8, 2)) + 1j * rng.normal(size=(8, 2))
    M = a @ b.conj().T
    s, _, full = kept_sigma(M, 4)
    exact = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(s[:2], exact[:2], rtol=1e-12)
    assert not full
