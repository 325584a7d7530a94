"""Continuous-batching job server for ESCG simulations on one GPU.

Requests (lattice side L, species S with circulant dominance K, mobility,
MCS budget, seed) arrive over time.  The scheduler admits queued jobs in
arrival order while the job's device footprint fits the HBM budget and a
slot is free, keeps every admitted job's lattice resident on the device,
and runs iterations: each iteration advances every active job by a chunk of
MCS sized to a common amount of work, then retires finished jobs.  Jobs that
arrive while an iteration runs join at the next iteration boundary.

Work within an iteration overlaps on the device: all active jobs small
enough for one workgroup's LDS advance together in one persistent batched
launch (one workgroup per job, on a share of the CUs), while the larger
jobs advance together on a second stream in persistent launches that each
hold the tiles of several jobs (every tile resident in LDS for the job's
whole chunk, halos exchanged within its job) on the remaining CUs.
Because every random draw
is keyed by (seed, replica, MCS, pass, site), a job's result does not depend
on its co-runners, on chunking or on admission time: it is byte-identical to
the job run alone.

The executor interface (alloc / advance / collect / free) keeps the
scheduler testable with a CPU executor and an injected clock.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class JobState:
    req: object                    # workloads.Request
    done_mcs: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    handle: object = None          # executor-owned device state
    result: Optional[np.ndarray] = None  # final counts[0..S]
    failed: str = ""

    @property
    def footprint(self) -> int:
        return footprint_bytes(self.req.L)


def footprint_bytes(L: int) -> int:
    """Device bytes a job holds while admitted: its lattice plus the
    ping-pong lattice of the per-MCS tiled path."""
    return 2 * L * L + 4096


@dataclass
class ServerConfig:
    hbm_budget: int = 64 << 30     # bytes of device memory for job state
    max_active: int = 512          # slots
    # Chunk of a job per iteration: work_per_iter site-updates, clamped to
    # [min_chunk, max_chunk] MCS.  The cap keeps iterations short when small
    # lattices would take thousands of MCS, so large jobs are not held
    # behind them.  On the serving mix (L in {100..1600}), measured as
    # (p50, p99 at 200 jobs/s; p50, p99 at 400 jobs/s; jobs/s at
    # saturation): 1e9 / 500: 0.085 s, 0.22 s; 0.15 s, 0.47 s; 489.
    # 2e9 / 1000: 0.094 s, 0.17 s; 0.16 s, 0.44 s; 397.  3e9 / 1500: 0.11 s,
    # 0.19 s; 0.18 s, 0.49 s; 503.  4e8 / 500: 0.16 s, 0.72 s; 0.50 s,
    # 2.5 s; 385.
    work_per_iter: float = 1e9     # site-updates per job per iteration
    min_chunk: int = 8             # MCS
    max_chunk: int = 500           # MCS


@dataclass
class Stats:
    latencies: List[float] = field(default_factory=list)
    completed: int = 0
    failed: int = 0
    iterations: int = 0
    peak_active: int = 0
    peak_footprint: int = 0
    site_updates: float = 0.0
    wall: float = 0.0

    def summary(self) -> Dict[str, float]:
        lat = np.asarray(self.latencies) if self.latencies else np.zeros(1)
        return {
            "completed": self.completed,
            "failed": self.failed,
            "jobs_per_s": self.completed / self.wall if self.wall else 0.0,
            "site_updates_per_s": self.site_updates / self.wall
            if self.wall else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "iterations": self.iterations,
            "peak_active": self.peak_active,
            "peak_footprint_bytes": self.peak_footprint,
            "wall_s": self.wall,
        }


class Scheduler:
    """Admission, iteration and retirement; device work goes through the
    executor.  `clock()` returns seconds; arrivals are relative to the start
    of run()."""

    def __init__(self, executor, config: ServerConfig = ServerConfig(),
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.cfg = config
        self.clock = clock
        self.sleep = sleep

    def chunk_for(self, job: JobState) -> int:
        c = int(self.cfg.work_per_iter / float(job.req.L) ** 2)
        c = max(self.cfg.min_chunk, min(self.cfg.max_chunk, c))
        return min(c, job.req.mcs - job.done_mcs)

    def run(self, requests) -> (Stats, Dict[int, JobState]):
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = deque(reqs)
        queue: deque = deque()
        active: List[JobState] = []
        jobs: Dict[int, JobState] = {}
        st = Stats()
        used = 0
        t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                r = pending.popleft()
                js = JobState(req=r)
                jobs[r.job_id] = js
                queue.append(js)
            # admission: arrival order, no overtaking
            while queue and len(active) < self.cfg.max_active:
                js = queue[0]
                if js.footprint > self.cfg.hbm_budget:
                    queue.popleft()
                    js.failed = "footprint exceeds the HBM budget"
                    st.failed += 1
                    continue
                if used + js.footprint > self.cfg.hbm_budget:
                    break
                queue.popleft()
                try:
                    js.handle = self.ex.alloc(js.req)
                except Exception as e:  # invalid job: isolate it
                    js.failed = f"rejected: {e}"
                    st.failed += 1
                    continue
                js.t_admit = self.clock() - t0
                used += js.footprint
                active.append(js)
            st.peak_active = max(st.peak_active, len(active))
            st.peak_footprint = max(st.peak_footprint, used)
            if not active:
                if pending:
                    wait = pending[0].arrival_s - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue
            work = [(js, self.chunk_for(js)) for js in active]
            try:
                self.ex.advance([(js.handle, js.req, js.done_mcs, n)
                                 for js, n in work])
            except Exception as e:  # executor failure: fail this iteration's
                for js, _ in work:  # jobs, keep serving the others
                    js.failed = f"executor: {e}"
                    st.failed += 1
                    self.ex.free(js.handle)
                    used -= js.footprint
                active = []
                continue
            st.iterations += 1
            still = []
            for js, n in work:
                js.done_mcs += n
                st.site_updates += float(js.req.L) ** 2 * n
                if js.done_mcs >= js.req.mcs:
                    js.result = self.ex.collect(js.handle, js.req)
                    js.t_done = self.clock() - t0
                    st.latencies.append(js.t_done - js.req.arrival_s)
                    st.completed += 1
                    self.ex.free(js.handle)
                    used -= js.footprint
                else:
                    still.append(js)
            active = still
        st.wall = self.clock() - t0
        return st, jobs


class DeviceExecutor:
    """Runs jobs on the current GPU through the C ABI."""

    def __init__(self, torch, escg, n_streams: int = 4,
                 keep_lattices: bool = False,
                 small_share: Optional[float] = 0.25,
                 large_route: str = "persistent",
                 small_L: Optional[int] = None, light_jobs: int = 128):
        self.torch = torch
        self.escg = escg
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.batch_stream = torch.cuda.Stream()
        self.small_max = {}
        self.keep = keep_lattices
        self.final_lattices: Dict[int, np.ndarray] = {}
        self.cus = torch.cuda.get_device_properties(0).multi_processor_count
        # share of the CUs the small jobs' batch may hold while large jobs
        # run beside it (None: the small jobs' share of the iteration's
        # site-updates, which measured slower on the serving mix: 456
        # against 482 jobs/s at saturation); the large jobs' persistent
        # launches get the rest, so both kernels' workgroups are resident
        # together
        self.small_share = small_share
        self.large_route = large_route  # "persistent" or "tiled" (per MCS)
        # Largest side advanced whole in one workgroup's LDS (beside the
        # LDS limit): None = adaptive: 256 while at most light_jobs jobs are
        # active (an L = 400 lattice then runs faster as tiles on a few CUs:
        # on the serving mix at 200 jobs/s p50 0.07 s and p99 0.17 s against
        # 0.14 s and 0.29 s), no further limit when more are (one workgroup
        # per small job packs the GPU better: 482 against 458 jobs/s at
        # saturation).
        self.small_L = small_L
        self.light_jobs = light_jobs
        self._limit = small_L if small_L is not None else 1 << 30
        self._inflight = None  # event of the last queued iteration
        self._res = []

    def _params(self, req):
        return self.escg.Params(L=req.L, S=req.S,
                                dom=self.escg.circulant_dom(req.S, req.K),
                                ex=req.ex, sel=1.0, rep=1.0, seed=req.seed,
                                replica=0)

    def _tuned(self, p, kernel):
        """p with the autotuned launch choices of `kernel` for its side
        (tile shape of the multi-job or single-job persistent kernel);
        unchanged if none are cached."""
        from paper_2508_16639_amd import autotune
        return autotune.apply(self.torch, p.with_launch(tile=None), kernel)

    def share(self, small, large) -> float:
        """Share of the CUs for the small jobs: fixed, or their share of the
        iteration's site-updates (a small job runs on one workgroup, a large
        job's tiles on one CU each, at about the same rate per CU)."""
        if self.small_share is not None:
            return self.small_share
        ws = sum(float(r.L) ** 2 * n for _, r, _, n in small)
        wl = sum(float(r.L) ** 2 * n for _, r, _, n in large)
        return ws / (ws + wl) if ws + wl > 0 else 0.5

    def is_small(self, req) -> bool:
        """Whole lattice fits one workgroup's LDS beside the rule tables of
        its kernel instantiation (S <= 7 or S > 7; the two run as separate
        batches, so an S > 7 job never shrinks the S <= 7 limit) and is not
        above small_L (larger lattices advance faster, per MCS, as tiles on
        several CUs)."""
        if req.S not in self.small_max:
            self.small_max[req.S] = self.escg.batch_max_L(req.S)
        return req.L <= min(self.small_max[req.S], self._limit)

    def alloc(self, req):
        p = self._params(req)
        self.escg.thresholds(p)  # validates rates
        lat = self.torch.empty(req.L * req.L, dtype=self.torch.uint8,
                               device="cuda")
        self.escg.init(p, lat)  # current stream; work streams wait on it
        return {"p": p, "lat": lat}

    def advance(self, work):
        try:
            self._advance(work)
        except Exception:
            # work may already be enqueued on the side streams: let it end
            # before the caller frees (and the allocator reuses) lattices
            self.torch.cuda.synchronize()
            raise

    def _advance(self, work):
        torch, escg = self.torch, self.escg
        if self.small_L is None:
            self._limit = 256 if len(work) <= self.light_jobs else 1 << 30
        small = [(h, r, m0, n) for h, r, m0, n in work if self.is_small(r)]
        large = [(h, r, m0, n) for h, r, m0, n in work if not self.is_small(r)]
        cur = torch.cuda.current_stream()
        done = []
        self.batch_stream.wait_stream(cur)
        for s in self.streams:
            s.wait_stream(cur)
        small_wgs = 0
        if small and large:
            small_wgs = min(len(small), self.cus - 1,
                            max(1, round(self.cus * self.share(small, large))))
        # small jobs: one persistent batched launch per kernel instantiation
        # (S <= 7 and S > 7 tables), one after the other on the batch stream
        res_keep = []
        for group in ([w for w in small if w[1].S <= 7],
                      [w for w in small if w[1].S > 7]):
            if not group:
                continue
            if small_wgs:
                group[0] = (dict(group[0][0],
                                 p=group[0][0]["p"].with_launch(
                                     max_wgs=small_wgs)),) + group[0][1:]
            # lattices live in separate tensors: offsets from the lowest
            base = min(h["lat"].data_ptr() for h, _, _, _ in group)
            top = max(h["lat"].data_ptr() + r.L * r.L for h, r, _, _ in group)
            view = _DevView(base, top - base)
            offs = [h["lat"].data_ptr() - base for h, _, _, _ in group]
            res = torch.empty(len(group) * escg.BATCH_RESULT_WORDS,
                              dtype=torch.int32, device="cuda")
            with torch.cuda.stream(self.batch_stream):
                escg.batch_run([h["p"] for h, _, _, _ in group], offs, view,
                               [n for _, _, _, n in group],
                               escg.STOP_NONE, False, res,
                               mcs0=[m0 for _, _, m0, _ in group])
            res_keep.append(res)
        if small:
            with torch.cuda.stream(self.batch_stream):
                ev = torch.cuda.Event()
                ev.record()
                done.append(ev)
            # alive until the iteration completes (the host runs up to one
            # iteration ahead, so keep the last two iterations' buffers)
            self._res = (self._res + [res_keep])[-2:]
        # large jobs with a tile plan advance together in persistent
        # launches of several jobs each (or one launch per MCS for all of
        # them with large_route "tiled"); any others run alone on the
        # remaining streams
        tiled = [w for w in large if w[1].L % 8 == 0 and w[1].L >= 16]
        alone = [w for w in large if not (w[1].L % 8 == 0 and w[1].L >= 16)]
        if len(tiled) == 1 and not small and not alone:
            # a lone large job has the GPU to itself: the persistent kernel
            # (all of this iteration's MCS in one cooperative launch) is
            # about twice as fast per MCS as one launch per MCS
            alone, tiled = tiled, []
        if tiled:
            kern = "multi" if self.large_route == "persistent" else "step"
            ps = [self._tuned(h["p"], kern) for h, _, _, _ in tiled]
            cap = self.cus - small_wgs
            ps[0] = ps[0].with_launch(
                route=self.large_route,
                max_wgs=cap if small_wgs else 0)
            with torch.cuda.stream(self.streams[0]):
                escg.step_batch(ps,
                                [h["lat"] for h, _, _, _ in tiled],
                                [m0 for _, _, m0, _ in tiled],
                                [n for _, _, _, n in tiled])
                ev = torch.cuda.Event()
                ev.record()
                done.append(ev)
        others = self.streams[1:] or self.streams
        # one launch per MCS for these too while other launches run: a
        # cooperative persistent launch would wait for CUs that they hold
        lone = len(alone) == 1 and not small and not tiled
        for i, (h, r, m0, n) in enumerate(alone):
            s = others[i % len(others)]
            p = (self._tuned(h["p"], "persistent") if lone
                 else h["p"].with_launch(route="tiled"))
            with torch.cuda.stream(s):
                escg.step_mcs(p, h["lat"], m0, n, None)
                ev = torch.cuda.Event()
                ev.record()
                done.append(ev)
        for ev in done:
            cur.wait_event(ev)
        # No host synchronisation per iteration: the next iteration's
        # streams wait for this one through the current stream, and so does
        # every later use of a freed lattice's memory (allocated on the
        # current stream).  The host runs at most one iteration ahead: it
        # waits for the previous iteration here while this one is queued.
        # Results are read by collect(), which synchronises its own copy.
        ev = torch.cuda.Event()
        ev.record(cur)
        if self._inflight is not None:
            self._inflight.synchronize()
        self._inflight = ev

    def collect(self, h, req):
        cnt = self.torch.empty(req.S + 1, dtype=self.torch.int32,
                               device="cuda")
        self.escg.densities(h["p"], h["lat"], cnt)
        if self.keep:
            self.final_lattices[req.job_id] = h["lat"].cpu().numpy().copy()
        return cnt.cpu().numpy().view(np.uint32).copy()

    def free(self, h):
        h.clear()


class _DevView:
    """A raw device span presented to escg.batch_run as a uint8 tensor-like
    object (pointer + size); the spans of the jobs inside are disjoint
    tensors owned by the executor."""

    def __init__(self, ptr: int, nbytes: int):
        import torch
        self._ptr = ptr
        self._n = nbytes
        self.is_cuda = True
        self.dtype = torch.uint8

    def data_ptr(self):
        return self._ptr

    def numel(self):
        return self._n

    def is_contiguous(self):
        return True


def plain_serving(torch, escg, requests, clock=time.perf_counter,
                  sleep=time.sleep):
    """Baseline: one job at a time in arrival order, each with the best
    single-job path (init, all MCS, counts, synchronise)."""
    st = Stats()
    t0 = clock()
    for r in sorted(requests, key=lambda r: r.arrival_s):
        now = clock() - t0
        if r.arrival_s > now:
            sleep(r.arrival_s - now)
        p = escg.Params(L=r.L, S=r.S, dom=escg.circulant_dom(r.S, r.K),
                        ex=r.ex, seed=r.seed)
        lat = torch.empty(r.L * r.L, dtype=torch.uint8, device="cuda")
        cnt = torch.empty(r.S + 1, dtype=torch.int32, device="cuda")
        escg.init(p, lat)
        escg.step_mcs(p, lat, 0, r.mcs, None)
        escg.densities(p, lat, cnt)
        torch.cuda.synchronize()
        st.latencies.append(clock() - t0 - r.arrival_s)
        st.completed += 1
        st.site_updates += float(r.L) ** 2 * r.mcs
    st.wall = clock() - t0
    return st


def bench_serving(torch, escg, workloads, n_jobs: int = 2000,
                  rates=(200.0, 400.0, 800.0), plain: bool = True):
    """The Poisson serving workload through the server at each arrival rate
    (the first is the workload's 200 jobs/s), at saturation (every request
    at t = 0: the server's capacity), and through plain one-at-a-time
    serving at the first rate, on the same GPU."""
    out = {"workload": f"{n_jobs} jobs, Poisson, S in {{3,5}}, "
                       "L in {100,200,400,800,1600}, M log-uniform "
                       "[1e-6,1e-3], MCS uniform [500,5000]",
           "by_rate": {}}
    base = None if rates else workloads.serving_requests(n=n_jobs)
    for rate in rates:
        reqs = workloads.serving_requests(n=n_jobs, rate_per_s=rate)
        st, _ = Scheduler(DeviceExecutor(torch, escg)).run(reqs)
        escg.async_status()
        out["by_rate"][f"{rate:g}"] = st.summary()
        if base is None:
            base = reqs
    reqs = [dataclasses.replace(r, arrival_s=0.0) for r in base]
    st, _ = Scheduler(DeviceExecutor(torch, escg)).run(reqs)
    escg.async_status()
    out["capacity"] = st.summary()
    if rates:
        out["server"] = out["by_rate"][f"{rates[0]:g}"]
    from paper_2508_16639_amd import autotune
    out["large_jobs_autotuned"] = {
        f"L={L},S<=7": autotune.lookup(torch, "multi", L, 3) is not None
        for L in sorted({r.L for r in base if r.L > 400})}
    if plain:
        pl = plain_serving(torch, escg, base).summary()
        out["plain"] = pl
        out["speedup_jobs_per_s"] = (out["server"]["jobs_per_s"] /
                                     pl["jobs_per_s"]
                                     if pl["jobs_per_s"] else None)
        out["capacity_vs_plain"] = (out["capacity"]["jobs_per_s"] /
                                    pl["jobs_per_s"]
                                    if pl["jobs_per_s"] else None)
        out["plain_note"] = ("plain serving is saturated at the first rate "
                             "(its jobs/s is its capacity); at higher rates "
                             "its queue only grows")
    return out
