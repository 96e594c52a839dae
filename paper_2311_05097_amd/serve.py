"""Continuous-batching job server for the coupled LBM on one GPU.

A stream of jobs (each: a domain, parameters and a step budget) arrives over
time.  The server keeps every admitted job's fields resident in GPU memory and
advances all of them in ticks, after which finished jobs are read out and
released and queued jobs are admitted as memory frees up.  Admission is by HBM
footprint: the sum of the resident jobs' workspaces stays under a byte budget.
Jobs whose fields become non-finite are detected after the tick
(``lbm_check``) and evicted as failed.

The resident jobs are packed into lanes, each an ``lbm_batch`` whose members'
workspaces together fit the GPU's last-level cache (``lane_bytes``); a tick
steps the lanes one after another on one stream, each with one fused launch
per time step over the tiles of all its members (replayed from a HIP graph).
One batch over everything would stream the whole resident set from HBM every
step; a lane's set stays in the cache for its steps.  Lanes on separate
streams, running together, measured 3-11% slower: together they no longer fit
the cache.

``run_solo`` is the baseline: the same stream processed one job at a time, each
with its own per-step launches (no batching, no graph).

Everything on the device runs in the library's kernels; this module only
schedules, through the C ABI.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbmgls
from .workloads import JobSpec


@dataclass
class JobResult:
    job_id: int
    side: int
    steps: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    status: str = "queued"         # done | failed
    mass_drift: float = math.nan
    phi: np.ndarray | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    mode: str
    jobs: list
    makespan: float
    ticks: int = 0

    def summary(self) -> dict:
        done = [j for j in self.jobs if j.status == "done"]
        failed = [j for j in self.jobs if j.status == "failed"]
        lat = np.array([j.latency for j in done]) if done else np.array([math.nan])
        lups = sum(j.side * j.side * j.steps for j in done)
        drift = [j.mass_drift for j in done if np.isfinite(j.mass_drift)]
        return {
            "mode": self.mode,
            "jobs_done": len(done),
            "jobs_failed": len(failed),
            "makespan_s": round(self.makespan, 3),
            "jobs_per_s": round(len(done) / self.makespan, 3) if self.makespan > 0 else None,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
            "glups": round(lups / self.makespan / 1e9, 2) if self.makespan > 0 else None,
            "max_rel_mass_drift": float(max(drift)) if drift else None,
            "ticks": self.ticks,
        }


def _sync():
    if lbmgls.DEVICE == "cuda":
        import torch
        torch.cuda.synchronize()


class Server:
    """Continuous batching over cache-sized lanes of lbm_batch."""

    def __init__(self, storage: str = "fp32", budget_bytes: int = 4 << 30, tick_steps: int = 500,
                 max_members: int = 128, tile: int = 0, keep_phi: bool = False,
                 job_overrides: dict | None = None, on_retire=None, lane_bytes: int | None = None):
        self.storage = storage
        self.budget = int(budget_bytes)
        self.tick = int(tick_steps)
        # tile 0: the autotuner's shape for this storage on a 1024^2 job, the
        # size of a lane (~1M nodes, its working set in the last-level cache);
        # one shape serves every member of a lane (lanes of 128^2 to 1024^2
        # jobs measured fastest in it: FP32 64x4, 4% above 64x8; FP16 64x8)
        self.tile = int(tile) if tile else _tuned_tile(1024, storage)
        self.keep_phi = keep_phi
        self.overrides = dict(job_overrides or {})
        self.on_retire = on_retire
        # lane capacity in workspace bytes; the part a step touches (both
        # population copies, history, statics; not the FP64 staging planes)
        # is ~0.8 of it, so these keep a lane's working set near the 256 MB
        # last-level cache (measured best of 96-320 MiB on a 64-job stream)
        if lane_bytes is None:
            lane_bytes = (320 << 20) if storage in ("fp16dev", "bf16dev") else (192 << 20)
        self.lane_bytes = int(lane_bytes)
        self.max_members = int(max_members)
        self.lanes: list = []     # [Batch, bytes resident in it]
        self.resident: list = []  # [JobResult, Domain, remaining, denominator, mass0, bytes, lane]
        self.used = 0

    def _new_lane(self):
        kw = dict(storage=self.storage, tile=self.tile, max_members=self.max_members,
                  max_tiles=self.max_members * (1024 * 1024 // (64 * 4)))
        if self.lanes:  # every lane on the first lane's stream: lanes run one after another
            kw["stream"] = self.lanes[0][0].stream
        self.lanes.append([lbmgls.Batch(**kw), 0])
        return self.lanes[-1]

    def _lane_for(self, nbytes: int):
        """The fullest lane the job fits in, else an empty one, else a new one."""
        fits = [ln for ln in self.lanes if ln[1] + nbytes <= self.lane_bytes]
        if fits:
            return max(fits, key=lambda ln: ln[1])
        empty = [ln for ln in self.lanes if ln[1] == 0]
        return empty[0] if empty else self._new_lane()

    def _footprint(self, spec: JobSpec) -> int:
        w = spec.workload(**self.overrides)
        return lbmgls.workspace_bytes(w.params, self.storage, self.tile), w

    def _admit(self, spec: JobSpec, res: JobResult, w, nbytes: int, now: float):
        lane = self._lane_for(nbytes)
        d = lane[0].domain(w.params, *w.arrays(), tile=self.tile)
        m0 = d.mass()
        lane[0].add(d)
        lane[1] += nbytes
        self.used += nbytes
        res.admitted = now
        self.resident.append([res, d, spec.steps, float(np.abs(w.phi).sum()), m0, nbytes, lane])

    def _retire(self, entry, now: float, status: str):
        res, d = entry[0], entry[1]
        if status == "done":
            res.mass_drift = abs(d.mass() - entry[4]) / entry[3]
            if self.keep_phi:
                res.phi = d.read()[0]
        res.status = status
        res.finished = now
        entry[6][0].remove(d)
        entry[6][1] -= entry[5]
        d.close()
        self.used -= entry[5]
        if self.on_retire is not None:
            self.on_retire(res)

    def run(self, jobs: list[JobSpec], realtime: bool = True) -> ServeStats:
        pending = sorted(jobs, key=lambda j: (j.arrival_s, j.job_id))
        results = {j.job_id: JobResult(j.job_id, j.side, j.steps, j.arrival_s) for j in jobs}
        sizes = {}
        t0 = time.perf_counter()
        ticks = 0
        while pending or self.resident:
            now = time.perf_counter() - t0
            # admit every arrived job that fits, in arrival order
            while pending and (not realtime or pending[0].arrival_s <= now):
                spec = pending[0]
                if spec.job_id not in sizes:
                    sizes[spec.job_id] = self._footprint(spec)
                nbytes, w = sizes[spec.job_id]
                if self.resident and self.used + nbytes > self.budget:
                    break
                pending.pop(0)
                self._admit(spec, results[spec.job_id], w, nbytes, time.perf_counter() - t0)
                del sizes[spec.job_id]
            if not self.resident:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival_s - now)))
                continue
            steps = {}
            for lane in self.lanes:
                # the lane's members in their order in the batch (admission order)
                members = [e for e in self.resident if e[6] is lane]
                if not members:
                    continue
                budget = [e[2] for e in members]
                n = min(self.tick, max(budget))
                lane[0].step(n, budget=budget)
                ticks += 1
                for e in members:
                    steps[id(e)] = min(n, e[2])
            _sync()
            now = time.perf_counter() - t0
            for e in list(self.resident):
                e[2] -= steps[id(e)]
                if not e[1].check():
                    self._retire(e, now, "failed")
                    self.resident.remove(e)
                elif e[2] == 0:
                    self._retire(e, now, "done")
                    self.resident.remove(e)
        makespan = time.perf_counter() - t0
        return ServeStats(f"batched-{self.storage}", list(results.values()), makespan, ticks)

    def close(self):
        for e in self.resident:
            e[6][0].remove(e[1])
            e[1].close()
        self.resident.clear()
        for lane in self.lanes:
            lane[0].close()
        self.lanes.clear()


def _tuned_tile(side: int, storage: str) -> int:
    from . import autotune
    return autotune.best_tile(JobSpec(0, side, 90.0, 10.0, 0).workload().params, storage)


def run_solo(jobs: list[JobSpec], storage: str = "fp32", tile: int = 0, check_every: int = 1000,
             realtime: bool = True, keep_phi: bool = False, job_overrides: dict | None = None,
             on_retire=None) -> ServeStats:
    """The plain per-job path: one job at a time, FIFO, per-step launches;
    tile 0: the autotuner's shape for each job's size."""
    overrides = dict(job_overrides or {})
    pending = sorted(jobs, key=lambda j: (j.arrival_s, j.job_id))
    out = []
    t0 = time.perf_counter()
    for spec in pending:
        now = time.perf_counter() - t0
        if realtime and spec.arrival_s > now:
            time.sleep(spec.arrival_s - now)
        res = JobResult(spec.job_id, spec.side, spec.steps, spec.arrival_s)
        w = spec.workload(**overrides)
        d = lbmgls.Domain(w.params, *w.arrays(), storage=storage, tile=tile or _tuned_tile(spec.side, storage))
        res.admitted = time.perf_counter() - t0
        m0 = d.mass()
        d.set_check(check_every)
        try:
            d.step(spec.steps)
            _sync()
            if not d.check():
                raise lbmgls.LbmError(-4, "non-finite at the end of the job")
            res.status = "done"
            res.mass_drift = abs(d.mass() - m0) / float(np.abs(w.phi).sum())
            if keep_phi:
                res.phi = d.read()[0]
        except lbmgls.LbmError:
            res.status = "failed"
        res.finished = time.perf_counter() - t0
        d.close()
        out.append(res)
        if on_retire is not None:
            on_retire(res)
    return ServeStats(f"solo-{storage}", out, time.perf_counter() - t0)
