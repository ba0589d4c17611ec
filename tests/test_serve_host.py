"""Host-side logic of the served form (no GPU): the request mix generator,
FIFO admission and latency percentiles."""
import math

import numpy as np

from workloads.configs import c5_case, c5_requests


def test_c5_request_mix():
    r = c5_requests()
    assert len(r) == 64
    arr = np.array([q["arrival"] for q in r])
    assert arr[0] == 0.0 and (np.diff(arr) >= 0).all()
    # exponential gaps, mean 0.05 s: the sample mean of 63 gaps is within 4 sigma
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 0.05) < 4 * 0.05 / math.sqrt(gaps.size)
    assert {q["n_r"] for q in r} <= {64, 128, 192, 256}
    assert {q["N"] for q in r} <= {2, 3, 4, 5}
    assert all(q["n_theta"] == 2 * q["n_r"] for q in r)
    assert all(0.05 <= q["h0"] <= 0.2 and 0.25 <= q["f"] <= 1.0 and 1e3 <= q["Re"] <= 1e4 for q in r)
    assert c5_requests() == r                      # seeded


def test_c5_case_sizes():
    q = dict(index=0, arrival=0.0, n_r=8, n_theta=16, N=3, h0=0.1, f=0.5, Re=2000.0, nsteps=10)
    c = c5_case(q)
    assert c.K == 4 * 8 * 8 and c.N == 3 and c.nsteps == 10
    assert c.motion["h0"] == 0.1 and abs(c.motion["omega"] - math.pi * 0.1) < 1e-15   # 2 pi f U, U = 0.1
    assert abs(c.tau - 0.1 / 2000.0) < 1e-18
    assert (c.face_tag == 1).sum() == 16 and (c.face_tag == 2).sum() == 16


def test_admit_fifo_no_overtaking():
    from paper_2607_00199_amd.serve import admit_fifo
    assert admit_fifo([3, 3, 3], 10) == 3
    assert admit_fifo([3, 8, 1], 10) == 1          # the 1 behind the 8 waits
    assert admit_fifo([], 10) == 0
    assert admit_fifo([11], 10) == 0
    assert admit_fifo([5, 5], 10) == 2


def test_latency_summary_nearest_rank():
    from paper_2607_00199_amd.serve import latency_summary
    s = latency_summary(range(1, 101))
    assert s["p50"] == 50 and s["p99"] == 99 and s["max"] == 100 and s["n"] == 100
    s = latency_summary([2.0])
    assert s["p50"] == s["p99"] == s["max"] == 2.0
    assert latency_summary([])["n"] == 0
