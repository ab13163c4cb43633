"""gtqa_bond_svd_noalloc (no device allocation, static scratch) against
gtqa_bond_svd on the same cores: two calls in a row, the second smaller, and
the size limit."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cores(rng, count, chi):
    n = 2 * chi
    out = []
    for _ in range(count):
        U, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
        V, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
        sig = rng.uniform(0.2, 0.9) ** np.arange(n)
        out.append((U * sig) @ V.conj().T)
    return np.stack(out)


@pytest.mark.parametrize("chi", [4, 8])
def test_noalloc_bond_svd_matches_the_allocating_entry_point(chi):
    from paper_2409_12240_amd import gtqa
    rng = np.random.default_rng(100 + chi)
    big = _cores(rng, gtqa.bond_svd_noalloc_max(chi), chi)
    small = _cores(rng, 37, chi)
    for cores in (big, small):
        ref, ref_sw = gtqa.bond_svd(chi, cores)
        got, got_sw = gtqa.bond_svd(chi, cores, noalloc=True)
        # same kernel and launch layout: identical results
        assert np.array_equal(got, ref)
        assert np.array_equal(got_sw, ref_sw)
        exact = np.linalg.svd(cores, compute_uv=False)
        np.testing.assert_allclose(got[:, :chi], exact[:, :chi], rtol=1e-11, atol=1e-13)


def test_noalloc_bond_svd_rejects_more_than_fits():
    from paper_2409_12240_amd import gtqa
    cap = gtqa.bond_svd_noalloc_max(4)
    assert cap > 1000
    with pytest.raises(gtqa.GtqaError) as ei:
        gtqa.bond_svd(4, np.zeros((cap + 1, 8, 8), dtype=np.complex128), noalloc=True)
    assert ei.value.code == gtqa.GTQA_ERR_ARG
    sig, sw = gtqa.bond_svd(4, np.zeros((0, 8, 8), dtype=np.complex128), noalloc=True)
    assert sig.shape == (0, 8)
