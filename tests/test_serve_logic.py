"""Host logic of the continuous-batching server (no GPU): admission by
workspace bytes under a budget, arrival order, per-job step budgets, eviction
of jobs that fail the finiteness check, retirement.  The device library is
replaced by a recording stand-in with the same interface; the GPU path itself
is tested in test_gpu_serving.py."""
import numpy as np
import pytest

from paper_2311_05097_amd import serve
from paper_2311_05097_amd import workloads as W


class FakeError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(msg)
        self.code = code


class FakeDomain:
    def __init__(self, lib, params, phi, *rest, **kw):
        self.lib = lib
        self.side = params["nx"]
        self.steps = 0
        self.bad = params["rho2"] < 1e-3  # stands for a job that goes non-finite
        self.closed = False

    def step(self, n):
        self.steps += n

    def set_check(self, every):
        pass

    def check(self):
        return not (self.bad and self.steps > 0)

    def mass(self):
        return 1.0

    def read(self):
        z = np.zeros((self.side, self.side))
        return z + self.steps, z, z, z

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self, lib, **kw):
        self.lib = lib
        self.members = []
        self.stream = kw.get("stream", object())  # lanes after the first share its stream
        self.lane_peak = 0
        lib.batches.append(self)

    def domain(self, params, *arrays, tile=0):
        return FakeDomain(self.lib, params, *arrays)

    def add(self, d):
        self.members.append(d)
        lane = sum(self.lib.footprint(m.side) for m in self.members)
        self.lane_peak = max(self.lane_peak, lane)
        used = sum(self.lib.footprint(m.side) for b in self.lib.batches for m in b.members)
        self.lib.peak = max(self.lib.peak, used)
        self.lib.order.append(d.side)

    def remove(self, d):
        self.members.remove(d)

    def step(self, n, budget=None):
        self.lib.ticks += 1
        for d, b in zip(self.members, budget):
            d.steps += min(n, b)

    def close(self):
        pass


class FakeLib:
    DEVICE = "cpu"
    LbmError = FakeError

    def __init__(self):
        self.peak = 0
        self.ticks = 0
        self.order = []
        self.batches = []

    @staticmethod
    def footprint(side):
        return side * side * 100

    def workspace_bytes(self, params, storage="fp32", tile=0):
        return self.footprint(params["nx"])

    def Batch(self, **kw):
        return FakeBatch(self, **kw)

    def Domain(self, params, *arrays, **kw):
        return FakeDomain(self, params, *arrays)


@pytest.fixture
def fake(monkeypatch):
    lib = FakeLib()
    monkeypatch.setattr(serve, "lbmgls", lib)
    return lib


def stream():
    sides = [64, 128, 64, 192, 128, 64, 64, 128]
    steps = [300, 120, 50, 260, 80, 500, 40, 90]
    jobs = [W.JobSpec(i, s, 60.0, 10.0, n, 0.0) for i, (s, n) in enumerate(zip(sides, steps))]
    jobs[3] = W.JobSpec(3, 192, 60.0, 5000.0, 260, 0.0)  # rho2 = 1/5000: fails its check
    return jobs


def test_server_admits_within_budget_in_arrival_order(fake):
    jobs = stream()
    budget = FakeLib.footprint(192) + FakeLib.footprint(128)
    srv = serve.Server(storage="fp32", budget_bytes=budget, tick_steps=100, tile=8, keep_phi=True)
    st = srv.run(jobs, realtime=False)
    srv.close()
    by = {j.job_id: j for j in st.jobs}
    assert fake.peak <= budget
    assert fake.order == [j.side for j in jobs]  # admitted in arrival order
    for j in jobs:
        r = by[j.job_id]
        if j.job_id == 3:
            assert r.status == "failed"
        else:
            assert r.status == "done"
            assert np.all(r.phi == j.steps)  # every job got exactly its step budget
            assert r.finished >= r.admitted >= r.arrival
    s = st.summary()
    assert s["jobs_done"] == 7 and s["jobs_failed"] == 1
    assert s["ticks"] == fake.ticks > 0


def test_server_admits_a_job_larger_than_the_budget_alone(fake):
    """A job whose footprint alone exceeds the budget is still served, by
    itself (nothing else resident), rather than blocking the queue."""
    jobs = [W.JobSpec(0, 64, 60.0, 10.0, 30, 0.0), W.JobSpec(1, 192, 60.0, 10.0, 30, 0.0),
            W.JobSpec(2, 64, 60.0, 10.0, 30, 0.0)]
    srv = serve.Server(storage="fp32", budget_bytes=FakeLib.footprint(128), tick_steps=10, tile=8)
    st = srv.run(jobs, realtime=False)
    assert all(j.status == "done" for j in st.jobs)
    assert fake.peak == FakeLib.footprint(192)


def test_solo_path_reports_failures_and_steps(fake):
    jobs = stream()
    st = serve.run_solo(jobs, storage="fp32", tile=8, keep_phi=True, realtime=False)
    by = {j.job_id: j for j in st.jobs}
    assert by[3].status == "failed"
    assert all(by[j.job_id].status == "done" and np.all(by[j.job_id].phi == j.steps)
               for j in jobs if j.job_id != 3)


def test_server_packs_jobs_into_cache_sized_lanes(fake):
    """Lanes hold at most lane_bytes of workspaces (a larger job gets a lane of
    its own), a job goes to the fullest lane it fits, all lanes share the first
    lane's stream, and every job still gets exactly its step budget."""
    jobs = stream()
    lane = FakeLib.footprint(128) + FakeLib.footprint(64)
    srv = serve.Server(storage="fp32", budget_bytes=10 * FakeLib.footprint(192), tick_steps=100, tile=8,
                       keep_phi=True, lane_bytes=lane)
    st = srv.run(jobs, realtime=False)
    srv.close()
    assert len(fake.batches) >= 3
    assert all(b.stream is fake.batches[0].stream for b in fake.batches)
    for b in fake.batches:
        assert b.lane_peak <= lane or b.lane_peak == FakeLib.footprint(192)
    by = {j.job_id: j for j in st.jobs}
    for j in jobs:
        if j.job_id != 3:
            assert by[j.job_id].status == "done" and np.all(by[j.job_id].phi == j.steps)
    assert st.summary()["ticks"] == fake.ticks
