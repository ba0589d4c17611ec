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


class _FakeLib:
    """Stand-in for the library calls the served loop makes: a batch whose
    steps take simulated time proportional to the active members' size; no
    GPU, no arithmetic.  Records what the loop did."""

    def __init__(self, sim, poisoned=(), unsupported=()):
        from paper_2607_00199_amd import _lib as L
        self.GbError, self.GB_FP32, self.make_params = L.GbError, L.GB_FP32, L.make_params
        self.sim, self.poisoned, self.unsupported = sim, set(poisoned), set(unsupported)
        self.max_used, self.admitted, self.live = 0, [], 0

    def gb_stream_create(self, device=0):
        return 1

    def gb_stream_destroy(self, s):
        pass

    def gb_ctx_create(self, device, stream):
        return object()

    def gb_ctx_destroy(self, ctx):
        pass

    def gb_batch_create(self, ctx, budget):
        return {"budget": budget, "used": 0, "members": {}, "next": 1}

    def gb_batch_destroy(self, b):
        pass

    def gb_batch_set_autotune(self, b, on):
        pass

    def gb_mesh_create(self, ctx, dim, N, vx, etov, period=None, face_tag=None):
        self.live += 1
        return {"K": len(etov), "dim": dim, "N": N}

    def gb_mesh_destroy(self, m):
        self.live -= 1

    def gb_set_motion(self, m, kind, p):
        pass

    def gb_mesh_sizes(self, m):
        Np = (m["N"] + 1) * (m["N"] + 2) // 2
        return m["K"], Np, 6, m["N"] + 1, 3

    def gb_mesh_nodes(self, m, dim):
        K, Np, *_ = self.gb_mesh_sizes(m)
        return np.zeros((K, dim, Np))

    def gb_solver_footprint(self, m, prm):
        return 1000 * m["K"]

    def gb_mesh_footprint(self, m):
        return 10 * m["K"]

    def gb_solver_create(self, m, prm):
        self.live += 1
        return {"mesh": m, "step": 0}

    def gb_solver_destroy(self, s):
        self.live -= 1

    def gb_state_set(self, s, q, t0=0.0):
        pass

    def gb_state_set_equilibrium(self, s, rho, u, offset=None, t0=0.0):
        pass

    def gb_equilibrium_moments(self, dim, c, rho, u):
        return np.zeros((6 if dim == 2 else 10, np.size(rho)))

    def gb_batch_add(self, b, s, dt, nsteps):
        if s["mesh"]["N"] in self.unsupported:
            raise self.GbError(7, "the batched form is not built for this element shape and precision")
        need = 1010 * s["mesh"]["K"]
        if b["used"] + need > b["budget"]:
            raise self.GbError(8, "busy")
        b["used"] += need
        self.max_used = max(self.max_used, b["used"])
        t = b["next"]
        b["next"] += 1
        b["members"][t] = {"s": s, "target": s["step"] + nsteps, "need": need}
        self.admitted.append(id(s))
        return t

    def gb_batch_info(self, b):
        return len(b["members"]), b["used"], b["budget"]

    def gb_batch_run(self, b, steps):
        for _ in range(steps):
            act = [m for m in b["members"].values() if m["s"]["step"] < m["target"]]
            self.sim[0] += 1e-6 * sum(m["s"]["mesh"]["K"] for m in act)
            for m in act:
                m["s"]["step"] += 1

    def gb_batch_poll(self, b, capacity=1024):
        done = [t for t, m in b["members"].items() if m["s"]["step"] >= m["target"]][:capacity]
        for t in done:
            b["used"] -= b["members"].pop(t)["need"]
        return done

    def gb_batch_class_count(self, b):
        return 0

    def gb_state_get(self, s, shape=None):
        if s["mesh"]["K"] in self.poisoned:
            raise self.GbError(5, "non-positive or NaN density latched on the device")
        return None, 0.0, s["step"]


def test_served_loop_scheduling_with_a_fake_library(monkeypatch):
    """Admission in arrival order without overtaking, the budget never
    exceeded, every request completed, a request whose footprint exceeds the
    whole budget rejected, and a request whose state fails reported as failed
    without stopping the others."""
    from paper_2607_00199_amd import serve as S
    from workloads import make_case
    sim = [0.0]
    sizes = [4, 8, 6, 12, 4, 8, 30, 6, 4, 10]          # quads per side; 30 is too large for the budget
    cases = [make_case("C1", n=n, N=2) for n in sizes]
    poisoned_K = cases[5].K                              # the request with n=8 at index 5 ...
    assert sum(c.K == poisoned_K for c in cases) == 2    # ... shares its size with index 1
    fake = _FakeLib(sim, poisoned={poisoned_K})
    monkeypatch.setattr(S, "L", fake)
    budget = 1010 * (2 * 12 * 12 + 2 * 8 * 8)           # two large-ish requests at once
    srv = S.Server(budget, steps_per_launch=3)
    reqs = [S.Request(index=i, arrival=0.01 * i, case=c, nsteps=5 + i) for i, c in enumerate(cases)]

    def sleep(dt):
        sim[0] += dt

    stats = srv.serve(reqs, clock=lambda: sim[0], sleep=sleep)
    assert fake.max_used <= budget
    assert stats["rejected"] == 1 and reqs[6].rejected
    assert stats["failed"] == 2 and reqs[1].error and reqs[5].error
    assert stats["completed"] == len(reqs) - 3
    ok = [r for r in reqs if not r.rejected and r.error is None]
    assert all(r.steps_done == r.nsteps for r in ok)
    assert all(r.t_done >= r.t_admit >= r.arrival for r in ok)
    # admitted in arrival order (the rejected one never admitted)
    order = [r.index for r in sorted((r for r in reqs if not r.rejected), key=lambda r: r.t_admit)]
    assert order == sorted(order)
    assert fake.live == 0                                # every mesh and solver released


def test_served_loop_request_the_batch_refuses_fails_alone(monkeypatch):
    """A request whose admission to the batch fails (a shape the batched
    kernel is not built for) is reported as failed, its solver and mesh are
    released, and every other request completes."""
    from paper_2607_00199_amd import serve as S
    from workloads import make_case
    sim = [0.0]
    cases = [make_case("C1", n=4, N=2), make_case("C1", n=4, N=5), make_case("C1", n=6, N=2)]
    fake = _FakeLib(sim, unsupported={5})
    monkeypatch.setattr(S, "L", fake)
    srv = S.Server(1 << 40, steps_per_launch=2)
    reqs = [S.Request(index=i, arrival=0.001 * i, case=c, nsteps=4) for i, c in enumerate(cases)]
    stats = srv.serve(reqs, clock=lambda: sim[0], sleep=lambda dt: sim.__setitem__(0, sim[0] + dt))
    assert stats["failed"] == 1 and reqs[1].error and "not built" in reqs[1].error
    assert stats["completed"] == 2 and all(reqs[i].steps_done == 4 for i in (0, 2))
    assert fake.live == 0


def test_served_loop_runs_to_the_next_completion_when_nobody_waits(monkeypatch):
    """With max_steps_per_launch set, the loop runs long stretches once every
    request has been admitted; every request still stops at its own step
    count and the budget is respected."""
    from paper_2607_00199_amd import serve as S
    from workloads import make_case
    sim = [0.0]
    cases = [make_case("C1", n=n, N=2) for n in (4, 6, 8, 5)]
    fake = _FakeLib(sim)
    runs = []
    orig = fake.gb_batch_run

    def run(b, steps):
        runs.append(steps)
        orig(b, steps)

    fake.gb_batch_run = run
    monkeypatch.setattr(S, "L", fake)
    srv = S.Server(1 << 40, steps_per_launch=2, max_steps_per_launch=40)
    reqs = [S.Request(index=i, arrival=0.0, case=c, nsteps=n) for i, (c, n) in enumerate(zip(cases, (50, 7, 23, 90)))]
    stats = srv.serve(reqs, clock=lambda: sim[0], sleep=lambda dt: sim.__setitem__(0, sim[0] + dt))
    assert stats["completed"] == 4
    assert all(r.steps_done == r.nsteps for r in reqs)
    assert max(runs) > 2 and max(runs) <= 40
    assert fake.live == 0
