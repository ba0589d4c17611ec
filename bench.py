"""Benchmark of the fused ALE Galerkin-Boltzmann SARK-4 path on one MI355X.

Workload: the 2D moving Taylor-Green vortex at scale -- a periodic square of
256 x 256 quads split into 131072 triangles, N = 4 (15 nodes), 6 fields,
sinusoidal mesh motion, Re 1000, Ma 0.05; FP32 with perturbation storage
q1 - rho0 (the reported value) and FP64 (reported beside it).

One step = one SARK-4 step: the per-vertex motion kernel, the four fused
stage kernels (geometry, volume, upwind surface, cubature relaxation, stage
combination) and the end-of-step vertex update.  Inputs are resident in HBM
before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  The metric is GDOF-stage/s = K_el * Np * NF * 4 *
steps / seconds / 1e9.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per stage launch of the FP32 2D N=4 stage kernel at 131072
# triangles, from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by kernels of
# known size (profiles/stage_kernel_c2_256_n4_mfma.md).  Reported only while
# the kernel and launch sources still hash to the digest they were measured
# with.
MEASURED_TRAFFIC = {
    "sources": ["paper_2607_00199_amd/csrc/gb_stage_mfma.hpp", "paper_2607_00199_amd/csrc/gb_stage_body.inc",
                "paper_2607_00199_amd/csrc/gb_stage.hpp", "paper_2607_00199_amd/csrc/gb_device.hpp",
                "paper_2607_00199_amd/csrc/gb_launch.hpp"],
    "sha256": "aa6654e126d360d89cff62b514f879b54946cb867177e9801faa058f91c66f1d",
    "K": 131072,
    "bytes_per_launch": 198233 * 1024,
}


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in MEASURED_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(K: int):
    if sources_digest() != MEASURED_TRAFFIC["sha256"] or K != MEASURED_TRAFFIC["K"]:
        return None
    return MEASURED_TRAFFIC["bytes_per_launch"]


def algorithmic_bytes_per_launch(K: int, Np: int, NF: int, dim: int, elem_bytes: int) -> float:
    """Bytes the stage kernel must move per launch: 15 state passes per
    SARK-4 step (3.75 per stage) of K*Np*NF values, plus per element the
    stage vertex coordinates ((dim+1)*dim FP64), the element's vertex ids and
    its face-neighbour ids ((dim+1) + (dim+1) int32)."""
    state = 3.75 * K * Np * NF * elem_bytes
    geom = K * ((dim + 1) * dim * 8 + 2 * (dim + 1) * 4)
    return state + geom


def run_gpu(precision_name: str, steps: int, warmup: int, n: int, graph: bool = True):
    import numpy as np
    import torch

    from paper_2607_00199_amd import _lib as L
    from paper_2607_00199_amd.session import Session
    from workloads import make_case

    prec = L.GB_FP32 if precision_name == "f32" else L.GB_FP64
    case = make_case("C2", n=n)

    def sync(sess):
        # the library's own HIP runtime is not torch's: wait on both
        L.gb_ctx_synchronize(sess.ctx)
        torch.cuda.synchronize()

    s = Session(case, precision=prec, device=0, stream=0)
    q0 = s.initial_state()
    s.set_state(q0)
    s.step(case.dt, warmup)
    sync(s)
    L.gb_solver_time_stages(s.solver, True)
    t0 = time.perf_counter()
    s.step(case.dt, steps)
    sync(s)
    el = time.perf_counter() - t0
    avg_ms, launches = L.gb_solver_stage_time(s.solver)
    by_kind = L.gb_solver_stage_time_by_kind(s.solver)
    L.gb_solver_time_stages(s.solver, False)
    q, t, nstep = s.get_state()
    # graph replay of the same step, timed separately
    gel = float("nan")
    if graph:
        s2 = Session(case, precision=prec, device=0, stream=0)
        s2.set_state(q0)
        s2.step(case.dt, warmup, graph=True)
        sync(s2)
        g0 = time.perf_counter()
        s2.step(case.dt, steps, graph=True)
        sync(s2)
        gel = time.perf_counter() - g0
        s2.close()
    K, Np, NF = s.K, s.Np, s.NF
    s.close()
    dof = K * Np * NF
    return {
        "case": case, "K": K, "Np": Np, "NF": NF, "dof": dof, "seconds": el, "graph_seconds": gel,
        "gdof_stage_s": dof * 4 * steps / el / 1e9,
        "graph_gdof_stage_s": dof * 4 * steps / gel / 1e9,
        "stage_avg_ms": avg_ms, "stage_launches": launches, "stage_ms_by_kind": [float(x) for x in by_kind],
        "q": q, "t": t, "steps_done": nstep,
    }


def run_other(name: str, steps: int, warmup: int) -> dict:
    """FP32 throughput of another workload: the 3D moving Taylor-Green vortex
    (663552 tetrahedra, N=3) or the plunging airfoil O-grid with walls, far
    field and sponge (262144 triangles, N=4)."""
    from paper_2607_00199_amd import _lib as L
    from paper_2607_00199_amd.serve import case_params
    from paper_2607_00199_amd.session import Session
    from workloads import make_case

    case = make_case(name)
    prm = case_params(case, L.GB_FP32)
    q_inf = list(prm.q_inf) if prm.sponge_sigma_max > 0 else None
    sponge = ((prm.sponge_cx, prm.sponge_cy, prm.sponge_r0, prm.sponge_r1, prm.sponge_sigma_max)
              if prm.sponge_sigma_max > 0 else None)
    s = Session(case, precision=L.GB_FP32, device=0, stream=0, q_inf=q_inf, sponge=sponge)
    s.set_state(s.initial_state())
    s.step(case.dt, warmup)
    L.gb_ctx_synchronize(s.ctx)
    L.gb_solver_time_stages(s.solver, True)
    t0 = time.perf_counter()
    s.step(case.dt, steps)
    L.gb_ctx_synchronize(s.ctx)
    el = time.perf_counter() - t0
    avg_ms, _ = L.gb_solver_stage_time(s.solver)
    K, Np, NF, dim = s.K, s.Np, s.NF, case.dim
    s.close()
    b = algorithmic_bytes_per_launch(K, Np, NF, dim, 4)
    return {"K": K, "N": case.N, "dim": dim, "dof": K * Np * NF, "steps": steps,
            "gdof_stage_s": round(K * Np * NF * 4 * steps / el / 1e9, 3), "stage_avg_ms": round(avg_ms, 5),
            "achieved_GBs": round(b / (avg_ms * 1e-3) / 1e9, 1),
            "frac": round(b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def energy_series(name: str, steps: int, every: int) -> dict:
    """Kinetic energy E_K and its rate eps = -dE_K/dt (Section 7.2) every
    `every` steps of an FP32 run of a workload, with the rate also estimated
    by centred differences of the E_K series as a consistency check."""
    from paper_2607_00199_amd import _lib as L
    from paper_2607_00199_amd.session import Session
    from workloads import make_case

    case = make_case(name)
    s = Session(case, precision=L.GB_FP32, device=0, stream=0)
    s.set_state(s.initial_state())
    t, ek, eps = [], [], []
    done = 0
    while True:
        e, r, _ = s.energy()
        t.append(done * case.dt)
        ek.append(e)
        eps.append(r)
        if done >= steps:
            break
        n = min(every, steps - done)
        s.step(case.dt, n)
        done += n
    s.close()
    fd = [None] + [-(ek[i + 1] - ek[i - 1]) / (t[i + 1] - t[i - 1]) for i in range(1, len(t) - 1)] + [None]
    return {"workload": name, "K": s.K, "N": case.N, "dim": case.dim, "dt": case.dt, "precision": "f32",
            "t": t, "E_K": ek, "eps": eps, "eps_centred_difference": fd}


def fp32_accuracy() -> dict:
    """Velocity of the FP32 path against the FP64 path (both on the GPU) at
    the final time of the accuracy workload: the 32x32-quad copy of the 2D
    moving Taylor-Green vortex (2048 triangles, N=4), 2000 SARK-4 steps."""
    import numpy as np

    from paper_2607_00199_amd import _lib as L
    from paper_2607_00199_amd.session import Session
    from workloads import make_case

    case = make_case("C2_small")
    vel = {}
    for prec in (L.GB_FP32, L.GB_FP64):
        s = Session(case, precision=prec, device=0, stream=0)
        s.set_state(s.initial_state())
        s.step(case.dt, case.nsteps)
        q, _, _ = s.get_state()
        s.close()
        vel[prec] = q[:, 1:3] / q[:, 0:1]
    u32, u64 = vel[L.GB_FP32], vel[L.GB_FP64]
    return {"workload": "32x32-quad copy of the 2D moving Taylor-Green vortex (2048 triangles, N=4), "
                        f"{case.nsteps} SARK-4 steps from the same initial state",
            "velocity_rel_err": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64)), "bound": 1e-5}


def host_cores() -> int:
    """Host cores this process may use (its CPU affinity), at most 16 (the
    host share of one GPU on a shared node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(seconds_budget: float = 15.0, copies: int = 1):
    """Time the oracle (unchanged) on a bounded sample of the workload: the
    32 x 32 copy of the same configuration (2048 triangles, N = 4), as many
    SARK-4 steps as fit the budget, each copy in a child process pinned to one
    thread.  With copies > 1, that many copies run at once on separate cores
    (the oracle itself is serial) and the rate is their aggregate."""
    code = r"""
import os, sys, time, json
sys.path.insert(0, %r)
from workloads import make_case
from oracle.mesh import Mesh
from oracle.rhs import Params
from oracle.solver import Solver
from oracle.motion import Motion
from oracle import gbsystem as gb
case = make_case("C2_small")
mot = dict(case.motion); kind = mot.pop("kind")
s = Solver(Mesh(2, case.N, case.vx, case.etov, case.period), Params(c=case.c, tau=case.tau), Motion(kind, **mot))
X = s.node_coords(); rho, u = case.macroscopic(X)
s.set_state(gb.equilibrium(2, rho, u, case.c).transpose(1, 0, 2).copy())
s.step(case.dt)
n = 0; t0 = time.perf_counter()
while time.perf_counter() - t0 < %f:
    s.step(case.dt); n += 1
el = time.perf_counter() - t0
dof = case.K * s.mesh.ref.Np * 6
print(json.dumps({"steps": n, "seconds": el, "K": case.K, "dof": dof, "gdof_stage_s": dof * 4 * n / el / 1e9}))
""" % (ROOT, seconds_budget)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                              text=True, env=env) for _ in range(copies)]
    res = []
    for pr in procs:
        out, err = pr.communicate(timeout=600)
        if pr.returncode != 0:
            return {"error": err[-500:]}
        res.append(json.loads(out.strip().splitlines()[-1]))
    agg = dict(res[0])
    agg["copies"] = copies
    agg["gdof_stage_s"] = sum(r["gdof_stage_s"] for r in res)
    agg["steps"] = sum(r["steps"] for r in res)
    return agg


def run_served(args, requests=None, steps=None) -> dict:
    """The served form on the request mix: Poisson arrivals of plunging-airfoil
    requests of mixed size and order, continuous batching under an HBM budget;
    then every request timed alone (graph replay) for the serial reference."""
    from paper_2607_00199_amd import serve as S
    from workloads.configs import c5_case, c5_requests

    specs = c5_requests(n=requests or args.requests, seed=1, nsteps=steps or args.served_steps)
    t0 = time.perf_counter()
    reqs = [S.Request(index=q["index"], arrival=q["arrival"], case=c5_case(q), nsteps=q["nsteps"]) for q in specs]
    print(f"served: {len(reqs)} request meshes generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    budget = int(args.budget_gib * (1 << 30)) if args.budget_gib > 0 else (1 << 50)
    srv = S.Server(budget, steps_per_launch=args.steps_per_launch, concurrency=args.concurrency,
                   autotune=not args.no_autotune, max_steps_per_launch=args.max_steps_per_launch)
    stats = srv.serve(reqs)
    srv.close()
    print(f"served: {stats['completed']} done in {stats['makespan_s']:.1f} s", file=sys.stderr, flush=True)
    serial_s = 0.0
    for r in reqs:
        serial_s += S.serial_rate(r, steps=args.serial_steps) * r.nsteps
    work = stats["dof_stages"]
    return {"stats": stats, "serial_seconds": serial_s, "serial_gdof_stage_s": work / serial_s / 1e9,
            "budget_bytes": budget, "requests": [
                {"K": r.case.K, "N": r.case.N, "arrival": round(r.arrival, 4), "admit": round(r.t_admit, 4),
                 "done": round(r.t_done, 4)} for r in reqs]}


def main_served(args):
    r = run_served(args)
    st = r["stats"]
    out = {
        "metric": "served aggregate GDOF-stage/s (continuous batching)",
        "value": round(st["gdof_stage_s"], 3), "unit": "GDOF-stage/s", "n_gpus": 1,
        "steps": args.served_steps, "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.requests} plunging-airfoil requests, Poisson arrivals 20/s, O-grid "
                               f"K in [16384, 262144], N in 2..5, {args.served_steps} SARK-4 steps each, FP32",
                   "budget_bytes": r["budget_bytes"], "steps_per_launch": args.steps_per_launch},
        "latency_s": st["latency_s"], "admission_wait_s": st["wait_s"], "makespan_s": round(st["makespan_s"], 3),
        "completed": st["completed"], "rejected": st["rejected"],
        "serial_plain_gdof_stage_s": round(r["serial_gdof_stage_s"], 3),
        "batched_vs_serial": round(st["gdof_stage_s"] / r["serial_gdof_stage_s"], 3),
        "classes": st["classes"],
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="quads per side (256 = the configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32 accuracy run on the 32x32-quad copy (e.g. under a kernel trace)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 512 MiB buffer three times (reference for HBM byte counters)")
    ap.add_argument("--all-configs", action="store_true",
                    help="also measure the 3D Taylor-Green and plunging-airfoil workloads (FP32)")
    ap.add_argument("--served", action="store_true",
                    help="run the served request mix instead (continuous batching, latency percentiles)")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--served-steps", type=int, default=1000)
    ap.add_argument("--budget-gib", type=float, default=0.0, help="admission budget (0 = the whole device)")
    ap.add_argument("--steps-per-launch", type=int, default=5)
    ap.add_argument("--serial-steps", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true", help="batched classes use the default launch tile")
    ap.add_argument("--max-steps-per-launch", type=int, default=64,
                    help="with no request waiting, run up to the next completion, at most this many steps")
    ap.add_argument("--concurrency", type=int, default=3,
                    help="streams on which large batch members run at once")
    ap.add_argument("--energy-series", metavar="WORKLOAD", default=None,
                    help="print the E_K / eps series of an FP32 run of WORKLOAD (e.g. C3) and exit")
    ap.add_argument("--series-every", type=int, default=25)
    ap.add_argument("--no-served", action="store_true",
                    help="skip the bounded served run appended to the default line")
    ap.add_argument("--served-requests-default", type=int, default=64,
                    help="requests of the bounded served run on the default line")
    ap.add_argument("--served-steps-default", type=int, default=1000,
                    help="steps per request of the bounded served run on the default line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.served:
        main_served(args)
        return
    if args.energy_series:
        steps = args.steps if "--steps" in sys.argv else 500
        print(json.dumps({"energy_series": energy_series(args.energy_series, steps, args.series_every)}))
        return

    import numpy as np

    if args.copy_calibration:
        # kernels of known size for the byte counters: a 512 MiB fill (writes
        # 512 MiB) and an elementwise scale of it (reads 512 MiB, writes 512 MiB)
        import torch
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    r32 = run_gpu("f32", args.steps, args.warmup, args.n, graph=not args.no_graph)
    r64 = None if args.no_fp64 else run_gpu("f64", args.steps, args.warmup, args.n, graph=not args.no_graph)

    case = r32["case"]
    K, Np, NF = r32["K"], r32["Np"], r32["NF"]
    bytes_launch = algorithmic_bytes_per_launch(K, Np, NF, 2, 4)
    achieved = bytes_launch / (r32["stage_avg_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(K)
    # the whole job as the library runs it: one step captured in a HIP graph
    # and replayed (gb_sark_step_graph), unless --no-graph; the eager figure
    # (one launch call per kernel, gb_sark_step) beside it
    graph = not args.no_graph
    secs = r32["graph_seconds"] if graph else r32["seconds"]
    out = {
        "metric": "GDOF-stage/s (FP32 perturbation storage; FP64 beside it)",
        "value": round(r32["dof"] * 4 * args.steps / secs / 1e9, 3),
        "unit": "GDOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D moving Taylor-Green vortex, periodic {args.n}x{args.n} quads -> {K} triangles, "
                               f"N={case.N} (Np={Np}), 6 fields, sin-product mesh motion A=0.05 T=1, Re 1000, Ma 0.05, "
                               f"dt={case.dt:.4e} (CFL 0.5), FP32 storage q1-rho0",
                   "K": K, "N": case.N, "dof": r32["dof"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": ("profile: rocprofv3 FETCH_SIZE and WRITE_SIZE of this kernel source, "
                                        "calibrated by kernels of known size, not measured in this run"
                                        if traffic is not None else
                                        "null: the kernel source changed since the counters were taken"),
                     "kernel": "stage_kernel<2,4,float,*> (4 stage kinds averaged)",
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": round(r32["stage_avg_ms"], 5),
                     "launches": r32["stage_launches"],
                     "avg_ms_by_stage": [round(x, 5) for x in r32["stage_ms_by_kind"]]},
        "launch": ("one SARK-4 step replayed from a HIP graph (gb_sark_step_graph)" if graph
                   else "eager launches (gb_sark_step)"),
        "eager": {"gdof_stage_s": round(r32["gdof_stage_s"], 3),
                  "ms_per_step": round(r32["seconds"] / args.steps * 1e3, 4)},
    }
    if r64 is not None:
        b64 = algorithmic_bytes_per_launch(K, Np, NF, 2, 8)
        a64 = b64 / (r64["stage_avg_ms"] * 1e-3) / 1e9
        u32 = r32["q"][:, 1:3] / r32["q"][:, 0:1]
        u64 = r64["q"][:, 1:3] / r64["q"][:, 0:1]
        out["fp64"] = {"gdof_stage_s": round(r64["gdof_stage_s"], 3),
                       "graph_gdof_stage_s": (None if args.no_graph else round(r64["graph_gdof_stage_s"], 3)),
                       "ms_per_step": round(r64["seconds"] / args.steps * 1e3, 4),
                       "stage_avg_ms": round(r64["stage_avg_ms"], 5),
                       "achieved_GBs": round(a64, 1), "frac": round(a64 / HBM_PEAK_GBS, 4)}
        out["fp32_accuracy"] = {} if args.no_accuracy else fp32_accuracy()
        # the same comparison on the timed runs above (warm-up plus timed
        # steps of the full-size workload; the bound is stated for the
        # accuracy workload's final time)
        out["fp32_accuracy"]["full_size_timed_run"] = {
            "steps": args.warmup + args.steps,
            "velocity_rel_err": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64))}
    if args.all_configs:
        out["other_configs"] = {"3D moving TGV, 663552 tets, N=3": run_other("C3", 20, 3),
                                "plunging airfoil O-grid, 262144 triangles, N=4": run_other("C4", 50, 5)}
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        out["cpu_baseline"] = {"value": round(cb.get("gdof_stage_s", float("nan")), 6), "unit": "GDOF-stage/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"FP64 numpy oracle, 32x32-quad copy of the workload (K={cb.get('K')}, N=4), "
                                         f"{cb.get('steps')} SARK-4 steps in {cb.get('seconds', 0):.1f} s, one thread"}
        ncores = host_cores()
        ca = cpu_baseline(copies=ncores)
        out["cpu_baseline_all_cores"] = {
            "value": round(ca.get("gdof_stage_s", float("nan")), 6), "unit": "GDOF-stage/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"{ncores} copies of the same sample at once, one per core (the oracle is serial), "
                      f"{ca.get('steps')} SARK-4 steps in total in about {ca.get('seconds', 0):.1f} s"}
    if not args.no_served:
        sr = run_served(args, requests=args.served_requests_default, steps=args.served_steps_default)
        st = sr["stats"]
        out["served"] = {
            "workload": f"{args.served_requests_default} plunging-airfoil requests of the served mix (Poisson "
                        f"arrivals 20/s, O-grid K in [16384, 262144], N in 2..5, FP32), "
                        f"{args.served_steps_default} SARK-4 steps each, continuous batching, whole-device budget",
            "completed": st["completed"], "failed": st["failed"], "rejected": st["rejected"],
            "latency_p50_s": st["latency_s"]["p50"], "latency_p99_s": st["latency_s"]["p99"],
            "latency_max_s": st["latency_s"]["max"],
            "aggregate_gdof_stage_s": round(st["gdof_stage_s"], 3),
            "serial_plain_gdof_stage_s": round(sr["serial_gdof_stage_s"], 3),
            "batched_vs_serial": round(st["gdof_stage_s"] / sr["serial_gdof_stage_s"], 3),
            "makespan_s": round(st["makespan_s"], 3)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
