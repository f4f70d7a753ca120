"""The serving executor's stepping thread (EngineStepper) on the CPU with a
test double for the batching engine: jobs advance one column per step, the
waiters return once their job is done, and an error in the stepping thread
reaches the waiters instead of leaving them waiting."""
import threading
import time

import pytest

from paper_2605_13209_amd.serve import EngineStepper


class FakeEngine:
    """Jobs of N columns; step() advances every unfinished job by one."""

    def __init__(self, fail_at_step=None):
        self.lock = threading.Lock()
        self.jobs = {}
        self.nsteps = 0
        self.fail_at_step = fail_at_step

    def add(self, N):
        with self.lock:
            j = len(self.jobs)
            self.jobs[j] = [0, N]
            return j

    def step(self):
        with self.lock:
            self.nsteps += 1
            if self.fail_at_step is not None and self.nsteps == self.fail_at_step:
                raise ValueError("planted step failure")
            active = [j for j, (c, N) in self.jobs.items() if c < N]
            fin = 0
            for j in active:
                self.jobs[j][0] += 1
                fin += self.jobs[j][0] == self.jobs[j][1]
        time.sleep(0.001)
        return len(active), fin

    def done(self, j):
        with self.lock:
            c, N = self.jobs[j]
            return c >= N


def test_jobs_from_many_threads_finish():
    eng = FakeEngine()
    st = EngineStepper(eng, timeout=30)
    out = []

    def worker(N):
        j = st.submit(lambda: eng.add(N))
        st.wait(j)
        out.append(N)

    ts = [threading.Thread(target=worker, args=(N,)) for N in (1, 5, 2, 64, 3, 17, 1, 8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=30)
    st.close()
    assert sorted(out) == sorted((1, 5, 2, 64, 3, 17, 1, 8))
    # the jobs shared steps: far fewer than the sum of their lengths
    assert eng.nsteps < 1 + 5 + 2 + 64 + 3 + 17 + 1 + 8


def test_step_error_reaches_the_waiters():
    eng = FakeEngine(fail_at_step=3)
    st = EngineStepper(eng, timeout=30)
    j = st.submit(lambda: eng.add(10))
    with pytest.raises(RuntimeError, match="batching engine stopped"):
        st.wait(j)
    with pytest.raises(RuntimeError, match="batching engine stopped"):
        st.submit(lambda: eng.add(2))
    st.close()


def test_wait_times_out():
    class Stuck(FakeEngine):
        def step(self):
            time.sleep(0.01)
            return 1, 0  # never finishes anything

    eng = Stuck()
    st = EngineStepper(eng, timeout=0.3)
    j = st.submit(lambda: eng.add(3))
    with pytest.raises(TimeoutError):
        st.wait(j)
    st.close()
