"""The allocation-free energy diagnostic (gb_energy_noalloc) against the
allocating form (gb_energy): the same kernels over a fixed device scratch
array, so the same state gives the same bits.  Two calls in a row, the second
on a smaller mesh (fewer workgroups, so fewer partial sums in the shared
array), and a 3D mesh after them."""
import pytest

from workloads import make_case

pytestmark = pytest.mark.gpu

from paper_2607_00199_amd import _lib as L  # noqa: E402
from paper_2607_00199_amd.session import Session  # noqa: E402


@pytest.mark.parametrize("prec", [L.GB_FP64, L.GB_FP32])
def test_energy_noalloc_matches_allocating_form(prec):
    cases = [make_case("C1", n=16), make_case("C1", n=4), make_case("C3", n=3, N=2)]
    sessions = []
    for case in cases:
        s = Session(case, precision=prec)
        s.set_initial_state()
        s.step(case.dt, 3)
        sessions.append(s)
    for s in sessions:
        first = L.gb_energy_noalloc(s.solver, 1.0)
        again = L.gb_energy_noalloc(s.solver, 1.0)
        ref = L.gb_energy(s.solver, 1.0)
        assert first == again == ref, (first, again, ref)
        assert ref[0] > 0.0 and ref[2] > 0.0
    for s in sessions:
        s.close()
