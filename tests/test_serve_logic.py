"""Host logic of the continuous-batching loop (CPU, with a fake pool).

The fake pool holds jobs up to a particle budget and a slot count, advances
every resident job by the chunk on each run, and reports finished jobs; the
tests check admission order, back-pressure (MD_EAGAIN), overlap of arrivals
with running work, and latency bookkeeping."""
import numpy as np

from paper_1411_3019_amd import serve
from paper_1411_3019_amd.md import Params


class FakePool:
    def __init__(self, budget, slots, log):
        self.budget, self.slots, self.log = budget, slots, log
        self.res = {}
        self.next = 0

    def admit(self, params, surface, surf, x, p, nsteps):
        used = sum(v["n"] for v in self.res.values())
        if len(self.res) >= self.slots or used + x.shape[0] > self.budget:
            return None
        jid = self.next
        self.next += 1
        self.res[jid] = dict(n=x.shape[0], left=nsteps, reported=False)
        self.log.append(("admit", jid, x.shape[0]))
        return jid

    def run(self, k):
        self.log.append(("run", tuple(sorted(self.res))))
        for v in self.res.values():
            v["left"] = max(0, v["left"] - k)

    def launch(self, k):
        # the fake's chunk is done at once; poll reports it
        self.run(k)

    def poll(self):
        out = [j for j, v in self.res.items() if v["left"] == 0 and not v["reported"]]
        for j in out:
            self.res[j]["reported"] = True
        return out

    def fetch(self, jid):
        return 0, {}

    def fetch_many(self, jids):
        return [self.fetch(j) for j in jids]

    def release(self, jid):
        del self.res[jid]

    def stats(self):
        return {}

    def close(self):
        pass


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _jobs(sizes, steps, arrivals):
    out = []
    for k, (n, s, a) in enumerate(zip(sizes, steps, arrivals)):
        out.append(serve.Job(k, a, Params(), "sphere", (0, 0, 0, 5.0), np.zeros((n, 3)), np.zeros((n, 3)), s))
    return out


def test_closed_loop_admission_and_backpressure():
    log = []
    jobs = _jobs([100, 200, 300, 400], [64, 32, 96, 32], [0, 0, 0, 0])
    clk = FakeClock()
    serve.serve(jobs, 0, 0, chunk=32, realtime=False, pool_factory=lambda: FakePool(600, 8, log), clock=clk,
                sleep=clk.sleep)
    admits = [e for e in log if e[0] == "admit"]
    # FIFO admission; the 400-particle job waits until room frees up
    assert [a[2] for a in admits] == [100, 200, 300, 400]
    first_run = next(e for e in log if e[0] == "run")
    assert first_run[1] == (0, 1, 2)
    # job 3 was admitted only after job 1 (32 steps) finished and was released
    i3 = log.index(("admit", 3, 400))
    assert any(e[0] == "run" for e in log[:i3])
    assert all(j.finished is not None and j.status == 0 for j in jobs)


def test_open_loop_arrivals_join_running_work():
    log = []
    clk = FakeClock()

    class TimedPool(FakePool):
        def run(self, k):
            super().run(k)
            clk.t += 0.01  # each chunk takes 10 ms

    jobs = _jobs([50, 50, 50], [320, 64, 64], [0.0, 0.015, 0.5])
    serve.serve(jobs, 0, 0, chunk=32, realtime=True, pool_factory=lambda: TimedPool(10 ** 6, 8, log), clock=clk,
                sleep=clk.sleep)
    runs = [e[1] for e in log if e[0] == "run"]
    # job 1 arrives while job 0 is running and shares its chunks
    assert (0, 1) in runs
    # the third job arrives after the first two finished: the loop idles (sleeps) until then
    assert jobs[2].admitted >= 0.5
    lat = [j.latency for j in jobs]
    assert all(v > 0 for v in lat)
    assert abs(jobs[1].latency - 0.025) < 0.011
    s = serve.summarize(jobs)
    assert s["jobs"] == 3 and s["failed"] == 0 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_oversized_job_is_reported():
    clk = FakeClock()
    jobs = _jobs([1000], [10], [0.0])
    try:
        serve.serve(jobs, 0, 0, realtime=False, pool_factory=lambda: FakePool(10, 8, []), clock=clk,
                    sleep=clk.sleep)
    except RuntimeError as e:
        assert "does not fit" in str(e)
    else:
        raise AssertionError("expected a RuntimeError")
