"""Continuous batching on the GPU: every served job's result is the same,
bit for bit, as the same job run alone (the serving layer changes when and
with whom a job runs, never what it computes)."""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_05097_amd import lbmgls
    lbmgls.lib()
    return lbmgls


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_served_jobs_equal_solo_runs(gpu, storage):
    from paper_2311_05097_amd import serve
    import torch
    spec = [(64, 60.0, 10.0, 300), (128, 120.0, 50.0, 220), (64, 90.0, 20.0, 500), (128, 45.0, 100.0, 150),
            (192, 75.0, 30.0, 120), (64, 135.0, 80.0, 260)]
    jobs = [W.JobSpec(i, s, th, r, n, 0.0) for i, (s, th, r, n) in enumerate(spec)]
    # a budget that holds one 192^2 job and one 128^2 job: admission binds
    budget = gpu.workspace_bytes(jobs[4].workload().params, storage, 8) + \
        gpu.workspace_bytes(jobs[1].workload().params, storage, 8)
    srv = serve.Server(storage=storage, budget_bytes=budget, tick_steps=100, tile=8, keep_phi=True)
    batched = srv.run(jobs, realtime=False)
    srv.close()
    torch.cuda.synchronize()
    solo = serve.run_solo(jobs, storage=storage, tile=8, keep_phi=True, realtime=False)
    a = {j.job_id: j for j in batched.jobs}
    b = {j.job_id: j for j in solo.jobs}
    for j in jobs:
        assert a[j.job_id].status == b[j.job_id].status == "done", j
        assert np.array_equal(a[j.job_id].phi, b[j.job_id].phi), j
        assert a[j.job_id].mass_drift == b[j.job_id].mass_drift
        print(f"\njob {j.job_id} {j.side}^2: identical, drift {a[j.job_id].mass_drift:.1e}")
    assert batched.ticks > 1


@pytest.fixture(scope="module")
def served_vs_oracle_jobs():
    """Two small jobs of the drop-on-slab stream (128^2 at 40 and 140 degrees,
    density ratios 30 and 90) and the oracle's phi after their step budgets."""
    from oracle.oracle import Oracle
    jobs = [W.JobSpec(0, 128, 40.0, 30.0, 600, 0.0), W.JobSpec(1, 128, 140.0, 90.0, 400, 0.0)]
    ref = {}
    for j in jobs:
        w = j.workload()
        o = Oracle(w.params, *w.arrays())
        o.step(j.steps)
        ref[j.job_id] = o.field("phi")
    return jobs, ref


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-5), ("fp16dev", 1e-3), ("bf16dev", 1e-3)])
def test_served_job_matches_oracle(gpu, served_vs_oracle_jobs, storage, tol):
    """A job served in a batch, compared with the FP64 oracle itself (not only
    with its solo run): the relative phi error in the 2-norm and the max-norm
    within the storage mode's bar (1e-5 for FP32, 1e-3 for the 16-bit
    deviation modes)."""
    from paper_2311_05097_amd import serve
    from parity import rel, relmax
    jobs, ref = served_vs_oracle_jobs
    srv = serve.Server(storage=storage, budget_bytes=1 << 30, tick_steps=100, tile=8, keep_phi=True)
    res = srv.run(jobs, realtime=False)
    srv.close()
    for j in res.jobs:
        assert j.status == "done", j
        e2, em = rel(j.phi, ref[j.job_id]), relmax(j.phi, ref[j.job_id])
        print(f"\nserved job {j.job_id} {storage}: phi error {e2:.2e} / {em:.2e}, mass drift {j.mass_drift:.1e}")
        assert e2 <= tol and em <= tol
