"""Admission policy of the request server, on the host with a simulated clock.

tests/sched_sim.cpp drives the policy header the server uses
(paper_2505_04431_amd/csrc/kc_sched.h) through an event simulation: jobs
arrive, workers pick them under a byte budget, keep their scratch, hold
results until released. No GPU is involved.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_sim")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall",
                           "-I", os.path.join(ROOT, "paper_2505_04431_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched_sim.cpp"), "-o", exe])

    def run(budget, workers, max_bypass, jobs):
        lines = ["%d %d %d %d" % (budget, workers, max_bypass, len(jobs))]
        for j in jobs:
            lines.append("%.6f %.6f %d %d %d %.6f" % j)
        r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
        out = r.stdout.split("\n")
        res = []
        for ln in out:
            f = ln.split()
            if not f:
                continue
            if f[0] == "peak":
                peak = int(f[1])
            elif f[0] == "stalls":
                run.stalls = int(f[1])
            else:
                res.append((float(f[1]), float(f[2]), int(f[3])))
        return res, peak

    run.stalls = 0
    return run


def random_jobs(seed, n, rate=1.0, max_scratch=10_000, exact=True, hold=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    jobs = []
    for i in range(n):
        scratch = int(rng.integers(100, max_scratch))
        actual = int(rng.integers(10, 1000))
        est = actual if exact else int(actual * rng.uniform(1.0, 3.0))
        jobs.append((t[i], float(rng.uniform(0.5, 3.0)), scratch, est, actual, hold))
    return jobs


def test_fifo_when_everything_fits(sim):
    jobs = random_jobs(1, 60)
    res, peak = sim(10**15, 3, 8, jobs)
    starts = [r[0] for r in res]
    assert starts == sorted(starts), "with room for everything the start order is the arrival order"
    # never more than 3 jobs at once
    ev = sorted([(s, 1) for s, e, w in res] + [(e, -1) for s, e, w in res])
    cur = top = 0
    for _, d in ev:
        cur += d
        top = max(top, cur)
    assert top <= 3


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_budget_respected(sim, seed):
    jobs = random_jobs(seed, 80, rate=3.0, exact=False)
    budget = 25_000
    res, peak = sim(budget, 4, 8, jobs)
    assert peak <= budget
    assert all(s >= j[0] - 1e-5 for (s, e, w), j in zip(res, jobs))


def test_bypass_bound(sim):
    # a large job arrives first while memory is tight; small jobs keep coming
    jobs = [(0.0, 5.0, 9_000, 500, 500, 0.1)]
    jobs.append((0.01, 2.0, 8_000, 500, 500, 0.1))     # takes most of the memory
    rng = np.random.Generator(np.random.PCG64(5))
    for i in range(40):
        jobs.append((0.02 + 0.05 * i, 0.3, int(rng.integers(100, 500)), 50, 50, 0.05))
    jobs.sort(key=lambda j: j[0])
    max_bypass = 4
    res, peak = sim(12_000, 4, max_bypass, jobs)
    for i, (s, e, w) in enumerate(res):
        later_first = sum(1 for m in range(i + 1, len(jobs)) if res[m][0] < s and jobs[m][0] >= jobs[i][0])
        assert later_first <= max_bypass, (i, later_first)
    assert peak <= 12_000


def test_scratch_is_held_only_while_running(sim):
    # four jobs with large scratch run side by side; then one job needs almost
    # the whole budget: it starts as soon as it arrives, since finished jobs
    # hold no scratch
    jobs = [(0.0 + 0.01 * i, 1.0, 3_000, 10, 10, 0.0) for i in range(4)]
    jobs.append((5.0, 1.0, 11_500, 100, 100, 0.0))
    res, peak = sim(12_000, 4, 8, jobs)
    assert res[-1][0] == pytest.approx(5.0)
    assert peak <= 12_000


def test_tighter_estimates_admit_more(sim):
    """Result reservations closer to the true size start jobs sooner
    (what a size predictor is for): mean latency drops, the budget holds."""
    base = random_jobs(7, 120, rate=4.0, max_scratch=3_000, exact=True, hold=2.0)
    loose = [(a, d, s, e * 8, act, h) for (a, d, s, e, act, h) in base]
    lat = []
    for jobs in (base, loose):
        res, peak = sim(20_000, 4, 8, jobs)
        assert peak <= 20_000
        lat.append(np.mean([e - j[0] for (s, e, w), j in zip(res, jobs)]))
    assert lat[0] < lat[1]


def test_held_results_beyond_the_budget_are_reported_not_waited_for(sim):
    """A client that waits for jobs in submission order and releases each
    result after its wait. Job 5 needs much more scratch than the others, so
    later small jobs pass it and finish; their results, held because the
    client is waiting for job 5, fill the budget. Without the stall report the
    queue would wait for ever (every worker idle, job 5 not admitted). With it the client releases what it holds and every job
    finishes; the ledger never passes the budget."""
    jobs = []
    for i in range(30):
        if i == 5:
            jobs.append((0.01 * i, 1.0, 2400, 300, 300, -1.0))
        else:
            jobs.append((0.01 * i, 0.2, 100, 300, 300, -1.0))
    res, peak = sim(3000, 2, 8, jobs)
    assert all(r[0] >= 0 for r in res)
    assert peak <= 3000
    assert sim.stalls >= 1


def test_no_stall_reports_when_results_are_released_in_time(sim):
    jobs = random_jobs(7, 80, hold=0.1)
    res, peak = sim(20_000, 3, 8, jobs)
    assert sim.stalls == 0
