"""Host-side checks of the library's table construction (no GPU).

  * gb_check_mesh_tables: the connectivity and blocked trace map the library
    builds for a mesh (periodic squares at every triangle order including
    N = 5, Kuhn cubes at every tetrahedron order, a walled O-grid, a
    tetrahedral box with far-field faces all round) have every index in
    range, are involutions on matched faces, the kernel's face-slot order
    (one face per lane quarter on tetrahedra) is a permutation of the face
    nodes, and the blocked copy equals the flat one in that order;
  * gb_check_batch_layout: the request-table layout of a batched launch class
    (members of the served mix's sizes, including the triangle order-5 FP64
    shape the batched form refuses) passes the checks the batch runs before
    every upload, and its dynamic LDS fits 160 KiB; a limit below it is
    reported;
  * the host setup code built with the address and undefined-behaviour
    sanitizers runs clean on the same meshes.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import kuhn_cube, ogrid_airfoil, periodic_square

L = pytest.importorskip("paper_2607_00199_amd._lib")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _meshes():
    out = []
    for N in (1, 2, 3, 4, 5):
        vx, etov, per, tag = periodic_square(5, seed=N, jitter=0.08)
        out.append((2, N, vx, etov, per, tag))
    for N in (1, 2, 3):
        vx, etov, per, tag = kuhn_cube(3)
        out.append((3, N, vx, etov, per, tag))
    vx, etov, per, tag = ogrid_airfoil(4, 16)
    out.append((2, 5, vx, etov, per, tag))
    vx, etov, _, _ = kuhn_cube(3, lo=-0.6, hi=1.4)
    out.append((3, 3, vx, etov, None, np.full((etov.shape[0], 4), 2, np.int8)))
    return out


def _lib_or_skip():
    try:
        L.load()
    except ImportError as ex:
        pytest.skip(str(ex))


@pytest.mark.parametrize("i", range(10))
def test_mesh_tables(i):
    _lib_or_skip()
    dim, N, vx, etov, per, tag = _meshes()[i]
    L.gb_check_mesh_tables(dim, N, vx, etov, per, tag)


def test_mesh_tables_report_bad_input():
    _lib_or_skip()
    vx, etov, per, tag = periodic_square(3, seed=0)
    bad = np.array(etov, copy=True)
    bad[4, 1] = vx.shape[0] + 7
    with pytest.raises(L.GbError):
        L.gb_check_mesh_tables(2, 3, vx, bad, per, tag)
    with pytest.raises(L.GbError) as ei:
        L.gb_check_mesh_tables(2, 3, vx, etov, None, None)     # boundary faces without tags
    assert ei.value.status == L.GB_ERR_MESH


@pytest.mark.parametrize("dim,N,prec", [(2, 5, 0), (2, 5, 1), (2, 4, 1), (3, 3, 1), (3, 3, 0), (3, 2, 1)])
def test_batch_layout_fits(dim, N, prec):
    _lib_or_skip()
    # served-mix member sizes: O-grids of n_r x 2 n_r quads, 64 members
    nr = np.array([64, 128, 192, 256] * 16)
    K = 4 * nr * nr
    nv = 2 * nr * (nr + 1)
    lds = L.gb_check_batch_layout(dim, N, prec, K, nv, 160 * 1024)
    assert 0 < lds <= 160 * 1024
    with pytest.raises(L.GbError) as ei:
        L.gb_check_batch_layout(dim, N, prec, K, nv, lds - 1)
    assert ei.value.status == L.GB_ERR_STATE


def _write_mesh(path, dim, N, vx, etov, per, tag):
    with open(path, "wb") as f:
        f.write(struct.pack("<iiqq", dim, N, vx.shape[0], etov.shape[0]))
        f.write(np.ascontiguousarray(vx, np.float64).tobytes())
        f.write(np.ascontiguousarray(etov, np.int32).tobytes())
        f.write(np.ascontiguousarray(np.zeros(dim) if per is None else per, np.float64).tobytes())
        f.write(struct.pack("<b", 0 if tag is None else 1))
        if tag is not None:
            f.write(np.ascontiguousarray(tag, np.int8).tobytes())


def test_host_setup_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "host_sanitize_driver.cpp"),
           os.path.join(ROOT, "paper_2607_00199_amd", "csrc", "host_ref.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    files = []
    for i, m in enumerate(_meshes()):
        p = str(tmp_path / f"mesh{i}.bin")
        _write_mesh(p, *m)
        files.append(p)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert r.stdout.count(": ok") == len(files)
