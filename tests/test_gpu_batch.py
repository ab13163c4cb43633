"""Mixed-chi batches (one pool per chi, each on its own stream, run
concurrently): every instance's result equals its single-instance run, and
the pools agree with the oracle."""

import numpy as np
import pytest

from oracle import gtqa as O
from synthetic import schedule_angles

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_mixed_chi_batch_matches_single_instances(precision):
    from paper_2409_12240_amd import gtqa
    from paper_2409_12240_amd.batch import MixedChiBatch, mixed_chi_instances
    insts, chis = mixed_chi_instances(count=10, n_half_range=(10, 40))
    T, dt = 4.0, 0.05
    res, wall, walls = MixedChiBatch(insts, chis, precision=precision).anneal(T, dt)
    assert set(walls) == {4, 8}
    tz, tx = schedule_angles(T, dt)
    dev = gtqa.TorchDevice()
    for i in (0, 1, 2, 3, 8, 9):
        st = gtqa.TrotterState(insts[i], device=dev, chi=chis[i], precision=precision)
        for k in range(tz.size):
            st.step(tz[k], tx[k])
        alone = st.readout()
        st.close()
        assert np.array_equal(alone["z"], res[i]["z"]), i
        assert np.array_equal(alone["x"], res[i]["x"]), i
        assert alone["energy"] == res[i]["energy"]
    # two instances against the oracle (FP64 1e-10, mixed 1e-3)
    for i in (0, 1):
        ost = O.init_state(insts[i], O.Options(chi=chis[i]))
        for k in range(tz.size):
            O.trotter_step(ost, tz[k], tx[k])
        dz = float(np.max(np.abs(res[i]["z"] - O.readout(ost)[0])))
        print(f"{precision} instance {i} (n={insts[i].n}, chi={chis[i]}): max |dz| vs oracle {dz:.2e}", flush=True)
        assert dz < (1e-10 if precision == "fp64" else 1e-3)
