"""C-ABI checks that need no GPU: the library loads, exports every function
include/gb.h declares, and its host-side reference operators (computed on the
CPU by the library's own setup code) agree with the oracle's, which are built by
a different route (product-Legendre basis in 40-digit arithmetic, quadrature
mass and face-mass matrices)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gb.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gb_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_00199_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2607_00199_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_error_strings(lib):
    from paper_2607_00199_amd import _lib
    assert "gfx950" in _lib.gb_version()
    with pytest.raises(_lib.GbError) as ei:
        _lib.gb_ref_operator(2, 4, 99)
    assert ei.value.status == _lib.GB_ERR_ARG
    with pytest.raises(_lib.GbError) as ei:
        _lib.gb_ref_operator(3, 9, 0)
    assert ei.value.status == _lib.GB_ERR_UNSUPPORTED


CASES = [(2, N) for N in range(1, 6)] + [(3, N) for N in range(1, 4)]


@pytest.mark.parametrize("dim,N", CASES)
def test_host_operators_match_oracle(dim, N):
    from oracle import refelem as R
    from paper_2607_00199_amd import _lib
    re_ = R.ref_element(dim, N)
    Np = re_.Np
    assert np.abs(_lib.gb_ref_operator(dim, N, 6).reshape(Np, dim) - re_.r).max() < 1e-14
    for a in range(dim):
        D = _lib.gb_ref_operator(dim, N, a).reshape(Np, Np)
        assert np.abs(D - re_.D[a]).max() < 1e-13 * max(1.0, np.abs(re_.D[a]).max())
    M = _lib.gb_ref_operator(dim, N, 7).reshape(Np, Np)
    assert np.abs(M - re_.M).max() < 1e-14
    # the library parametrises every face with reference measure 2, the
    # oracle with its true reference measure
    LIFT = _lib.gb_ref_operator(dim, N, 3).reshape(Np, -1)
    scale = np.repeat(re_.face_area / 2.0, re_.Nfp)
    ref = re_.LIFT / scale[None, :]
    assert np.abs(LIFT - ref).max() < 1e-13 * np.abs(ref).max()
    # cubature: same rule up to point order -> same projection of sampled data
    Ic = _lib.gb_ref_operator(dim, N, 4).reshape(-1, Np)
    Pc = _lib.gb_ref_operator(dim, N, 5).reshape(Np, -1)
    assert Ic.shape == re_.Icub.shape
    assert np.abs(Pc @ Ic - np.eye(Np)).max() < 1e-13
    rng = np.random.default_rng(dim * 10 + N)
    q = rng.normal(size=Np)
    f = lambda v: v * v / (3.0 + v)          # nonlinear map at the cubature points
    assert np.abs(Pc @ f(Ic @ q) - re_.Pcub @ f(re_.Icub @ q)).max() < 1e-12
