"""Write the FP64 oracle solution of the 32x32-quad copy of the 2D moving
Taylor-Green workload (2048 triangles, N=4, Re 1000, Ma 0.05, 2000 SARK-4
steps) used as the expected value of the FP32 accuracy test.

Calls only the oracle and the seeded input generators:

    python tests/golden/make_c2_small_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gbsystem as gb  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402
from oracle.motion import Motion  # noqa: E402
from oracle.rhs import Params  # noqa: E402
from oracle.solver import Solver  # noqa: E402
from workloads import make_case  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_small_oracle_2000.npz")


def main():
    case = make_case("C2_small")
    mot = dict(case.motion)
    kind = mot.pop("kind")
    s = Solver(Mesh(2, case.N, case.vx, case.etov, case.period), Params(c=case.c, tau=case.tau),
               Motion(kind, **mot))
    X = s.node_coords()
    rho, u = case.macroscopic(X)
    s.set_state(gb.equilibrium(2, rho, u, case.c).transpose(1, 0, 2).copy())
    t0 = time.time()
    for k in range(case.nsteps):
        s.step(case.dt)
        if (k + 1) % 200 == 0:
            print(f"step {k + 1}/{case.nsteps}  {time.time() - t0:.0f} s", flush=True)
    vel = gb.velocity(2, s.q.transpose(1, 0, 2), case.c)          # [2, K, Np]
    np.savez(OUT, velocity=vel, rho=s.q[:, 0], t=s.t, dt=case.dt, nsteps=case.nsteps, K=case.K, N=case.N,
             x_vertices=s.x)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
