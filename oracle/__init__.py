"""FP64 CPU oracle for the ALE Galerkin-Boltzmann nodal DG method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
reimplementation of the method, written from the paper (arXiv 2607.00199,
"A High-Order ALE DG Method for the Boltzmann Equation in Nearly Incompressible
Flows"), that the GPU library is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the GPU library (``paper_2607_00199_amd``) and neither imports the
other; both only read the seeded synthetic inputs in ``workloads``.

Everything is numpy float64.  Each module cites the passage of the paper it
follows.  Where the paper is silent, garbled or ambiguous the oracle takes the
reading listed in the design notes (flux sign convention, SARK row-sum typo,
cubature degree, 3D moment system); functions whose result is not pinned to
anything the paper or mathematics fixes say "parity unpinned" in their
docstring.

Parity-unpinned parts (see the individual docstrings):
  * the 3D 10-field moment system as a model of the paper's 3D runs (the
    paper only cites it; the tensor form taken restricts to the printed 2D
    system).  Its discretisation here is pinned to that tensor form by
    convergence against an independent spectral solution, and by its 2D
    restriction, spectrum, conservation and covariance.
The wall / far-field ghost states and the sponge layer are stand-ins for the
paper's wall treatment and perfectly matched layer, which it names without
giving their form: they are pinned by closed forms of their own definition
(a uniform state moving with a rigid wall, a free stream, a uniform offset
under the sponge), not by the paper.

Modules: refelem (reference operators), mesh (connectivity), gbsystem (moment
system), rhs (semi-discrete right-hand side), sark (time-integration
coefficients), motion (prescribed mesh motions), solver (SARK-4 steps on the
moving mesh), diagnostics (kinetic energy and its rate, wall force).
"""
