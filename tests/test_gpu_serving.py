"""Continuous-batching server on the GPU: completion under a tight HBM
budget (jobs must queue), and each job's result identical alone and in the
mix."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _alone(job, precision):
    from paper_2409_12240_amd import gtqa
    dev = gtqa.TorchDevice()
    pool = gtqa.Pool(chi=job.chi, precision=precision, max_vertices=job.instance.n, max_slots=1, device=dev)
    s = pool.admit(job.instance)
    tz, tx = job.schedule()
    for k in range(job.steps):
        pool.step([s], tz[k], tx[k])
    r = pool.readout(s)
    pool.close()
    return r


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_server_results_match_alone_and_budget_forces_queueing(precision):
    from paper_2409_12240_amd import gtqa
    from paper_2409_12240_amd.serve import Server, poisson_jobs
    jobs = poisson_jobs(seed=3000, count=10, rate_per_s=200.0, n_range=(40, 120), chis=(4, 8),
                        steps_range=(10, 30))
    # budget for about three resident jobs of the largest size
    fp = max(gtqa.gtqa_footprint_bytes(j.instance.n, j.instance.n_edges, j.chi,
                                       1 if precision == "mixed" else 0) for j in jobs)
    srv = Server(precision=precision, budget_bytes=3 * fp, max_vertices=4096, max_slots=16)
    out = srv.run(jobs, timeout_s=240)
    assert out["jobs"] == len(jobs)
    for j in out["completed"]:
        assert j.latency is not None and j.latency >= 0
        assert j.admitted >= j.arrival - 1e-9
    # with room for ~3 jobs some admissions must have waited
    assert any(j.admitted - j.arrival > 1e-4 for j in out["completed"])
    print(f"{precision}: p50 {out['p50_latency_s']*1e3:.1f} ms, p99 {out['p99_latency_s']*1e3:.1f} ms", flush=True)
    for j in sorted(out["completed"], key=lambda j: j.job_id)[:4]:
        alone = _alone(j, precision)
        assert np.array_equal(alone["z"], j.result["z"])
        assert np.array_equal(alone["x"], j.result["x"])
        assert alone["energy"] == j.result["energy"]
