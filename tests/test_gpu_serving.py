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
            (192, 75.0, 30.0, 120), (64, 135.0, 150.0, 260)]
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
