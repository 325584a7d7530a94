"""CPU stand-ins for the job server's device executor: the oracle (O2)
advances lattices in numpy, and a simulated clock charges each iteration a
duration proportional to its work."""
import numpy as np

import oracle as O


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class OracleExecutor:
    """Same interface as serve.DeviceExecutor; su_per_s sets the simulated
    speed.  fail_on: job ids whose alloc raises; fail_iter: iteration index
    at which advance raises."""

    def __init__(self, clock, su_per_s=1e9, fail_on=(), fail_iter=None):
        self.clock = clock
        self.rate = su_per_s
        self.fail_on = set(fail_on)
        self.fail_iter = fail_iter
        self.iter = 0
        self.live = {}
        self.max_live = 0
        self.final = {}

    def job(self, req):
        return O.Job(req.L, req.S, O.circulant_matrix(req.S, req.K), req.ex,
                     1.0, 1.0, seed=req.seed, replica=0)

    def alloc(self, req):
        if req.job_id in self.fail_on or req.L % 2:
            raise ValueError("invalid job")
        h = {"job": self.job(req), "id": req.job_id}
        h["lat"] = h["job"].init()
        self.live[req.job_id] = h
        self.max_live = max(self.max_live, len(self.live))
        return h

    def advance(self, work):
        self.iter += 1
        if self.fail_iter is not None and self.iter == self.fail_iter:
            raise RuntimeError("injected executor failure")
        su = 0.0
        for h, req, m0, n in work:
            O.o2_run(h["job"], h["lat"], m0, n, want_counts=False)
            su += float(req.L) ** 2 * n
        self.clock.t += su / self.rate

    def collect(self, h, req):
        self.final[req.job_id] = h["lat"].copy()
        return O.counts(h["lat"], req.L, req.S)

    def free(self, h):
        self.live.pop(h["id"], None)
