"""ctypes binding of the C ABI in include/gb.h (argument marshalling only).

Every computation runs in the HIP library ``libgb.so`` next to this file.  The
binding converts numpy arrays to plain pointers and raises ``GbError`` on any
status other than GB_OK.  It fails loudly when the library is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgb.so")

(GB_OK, GB_ERR_ARG, GB_ERR_MESH, GB_ERR_OOM, GB_ERR_DEVICE, GB_ERR_NONPHYSICAL, GB_ERR_STATE, GB_ERR_UNSUPPORTED,
 GB_ERR_BUSY) = range(9)
GB_FP64, GB_FP32 = 0, 1
GB_FLUX_SPLIT, GB_FLUX_RELATIVE = 0, 1
GB_FACE_INTERIOR, GB_FACE_WALL, GB_FACE_FARFIELD = 0, 1, 2
(GB_MOTION_NONE, GB_MOTION_SIN_PRODUCT_2D, GB_MOTION_TRIPLE_PRODUCT_3D, GB_MOTION_PLUNGE_BLEND_2D,
 GB_MOTION_VERTEX_ARRAY, GB_MOTION_FISH_3D) = range(6)

STATUS_NAMES = {0: "GB_OK", 1: "GB_ERR_ARG", 2: "GB_ERR_MESH", 3: "GB_ERR_OOM", 4: "GB_ERR_DEVICE",
                5: "GB_ERR_NONPHYSICAL", 6: "GB_ERR_STATE", 7: "GB_ERR_UNSUPPORTED", 8: "GB_ERR_BUSY"}


class GbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gb_motion(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 8)]


class gb_params(C.Structure):
    _fields_ = [("c", C.c_double), ("tau", C.c_double), ("precision", C.c_int), ("flux_mode", C.c_int),
                ("rho0", C.c_double), ("cubature_degree", C.c_int), ("q_inf", C.c_double * 10),
                ("sponge_cx", C.c_double), ("sponge_cy", C.c_double), ("sponge_r0", C.c_double),
                ("sponge_r1", C.c_double), ("sponge_sigma_max", C.c_double)]


_P = C.c_void_p
_i64 = C.c_int64
_dp = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "gb_last_error": (C.c_char_p, []),
    "gb_version": (C.c_char_p, []),
    "gb_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "gb_ctx_destroy": (None, [_P]),
    "gb_ctx_synchronize": (C.c_int, [_P]),
    "gb_stream_create": (C.c_int, [C.c_int, C.POINTER(_P)]),
    "gb_stream_destroy": (None, [_P]),
    "gb_mesh_create": (C.c_int, [_P, C.c_int, C.c_int, _i64, _dp, _i64, C.POINTER(C.c_int32), _dp,
                                 C.POINTER(C.c_int8), C.POINTER(_P)]),
    "gb_mesh_destroy": (None, [_P]),
    "gb_mesh_sizes": (C.c_int, [_P, C.POINTER(_i64), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "gb_ref_operator": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _i64, C.POINTER(_i64)]),
    "gb_check_mesh_tables": (C.c_int, [C.c_int, C.c_int, _i64, _dp, _i64, C.POINTER(C.c_int32), _dp,
                                       C.POINTER(C.c_int8)]),
    "gb_check_batch_layout": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_i64),
                                        C.POINTER(_i64), C.c_size_t, C.POINTER(C.c_size_t)]),
    "gb_mesh_nodes": (C.c_int, [_P, _dp]),
    "gb_mesh_vertices": (C.c_int, [_P, _dp]),
    "gb_set_motion": (C.c_int, [_P, C.POINTER(gb_motion)]),
    "gb_set_vertex_velocity": (C.c_int, [_P, _dp]),
    "gb_solver_create": (C.c_int, [_P, C.POINTER(gb_params), C.POINTER(_P)]),
    "gb_solver_destroy": (None, [_P]),
    "gb_solver_footprint": (C.c_int, [_P, C.POINTER(gb_params), C.POINTER(C.c_size_t)]),
    "gb_state_set": (C.c_int, [_P, _dp, C.c_double]),
    "gb_state_set_equilibrium": (C.c_int, [_P, _dp, _dp, _dp, C.c_double]),
    "gb_equilibrium_moments": (C.c_int, [C.c_int, C.c_double, _i64, _dp, _dp, _dp]),
    "gb_checkpoint_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "gb_checkpoint_save": (C.c_int, [_P, C.c_void_p, C.c_size_t]),
    "gb_checkpoint_load": (C.c_int, [_P, C.c_void_p, C.c_size_t]),
    "gb_energy": (C.c_int, [_P, C.c_double, _dp]),
    "gb_energy_noalloc": (C.c_int, [_P, C.c_double, _dp]),
    "gb_wall_force": (C.c_int, [_P, _dp]),
    "gb_state_get": (C.c_int, [_P, _dp, _dp, C.POINTER(_i64)]),
    "gb_rhs": (C.c_int, [_P, _dp, _dp]),
    "gb_sark_step": (C.c_int, [_P, C.c_double, _i64]),
    "gb_sark_step_graph": (C.c_int, [_P, C.c_double, _i64]),
    "gb_solver_time_stages": (C.c_int, [_P, C.c_int]),
    "gb_solver_stage_time": (C.c_int, [_P, _dp, C.POINTER(_i64)]),
    "gb_solver_stage_time_by_kind": (C.c_int, [_P, _dp]),
    "gb_mesh_footprint": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "gb_batch_create": (C.c_int, [_P, C.c_size_t, C.POINTER(_P)]),
    "gb_batch_destroy": (None, [_P]),
    "gb_batch_add": (C.c_int, [_P, _P, C.c_double, _i64, C.POINTER(C.c_uint64)]),
    "gb_batch_run": (C.c_int, [_P, _i64]),
    "gb_batch_poll": (C.c_int, [_P, C.POINTER(C.c_uint64), C.c_int, C.POINTER(C.c_int)]),
    "gb_batch_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "gb_batch_set_autotune": (C.c_int, [_P, C.c_int]),
    "gb_batch_set_concurrency": (C.c_int, [_P, C.c_int]),
    "gb_batch_class_count": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "gb_batch_class_info": (C.c_int, [_P, C.c_int, C.POINTER(_i64)]),
    "gb_batch_class_tile": (C.c_int, [_P, C.c_int, C.POINTER(_i64)]),
    "gb_tune_cache_save": (C.c_int, [C.c_char_p]),
    "gb_tune_cache_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    "gb_tune_cache_clear": (None, []),
}

_lib = None


def load():
    """Load libgb.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run python -m paper_2607_00199_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != GB_OK:
        raise GbError(status, load().gb_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- same-named calls

def gb_version() -> str:
    return load().gb_version().decode()


def gb_ctx_create(device: int = 0, stream: int = 0):
    out = _P()
    _check(load().gb_ctx_create(device, _P(stream or None), C.byref(out)))
    return out


def gb_ctx_destroy(ctx):
    load().gb_ctx_destroy(ctx)


def gb_ctx_synchronize(ctx):
    _check(load().gb_ctx_synchronize(ctx))


def gb_stream_create(device: int = 0) -> int:
    """A non-blocking stream of this library's HIP runtime (an integer
    handle for gb_ctx_create)."""
    out = _P()
    _check(load().gb_stream_create(device, C.byref(out)))
    return out.value or 0


def gb_stream_destroy(stream: int):
    load().gb_stream_destroy(_P(stream or None))


def gb_mesh_create(ctx, dim: int, N: int, vx, etov, period=None, face_tag=None):
    vx = _f64(vx)
    etov = np.ascontiguousarray(etov, dtype=np.int32)
    per = None if period is None else _f64(period)
    tag = None if face_tag is None else np.ascontiguousarray(face_tag, dtype=np.int8)
    out = _P()
    _check(load().gb_mesh_create(ctx, dim, N, vx.shape[0], _dptr(vx), etov.shape[0],
                                 etov.ctypes.data_as(C.POINTER(C.c_int32)),
                                 None if per is None else _dptr(per),
                                 None if tag is None else tag.ctypes.data_as(C.POINTER(C.c_int8)),
                                 C.byref(out)))
    return out


def gb_check_mesh_tables(dim: int, N: int, vx, etov, period=None, face_tag=None):
    """Host-only check of the library's connectivity and trace map for a mesh."""
    vx = _f64(vx)
    etov = np.ascontiguousarray(etov, dtype=np.int32)
    per = None if period is None else _f64(period)
    tag = None if face_tag is None else np.ascontiguousarray(face_tag, dtype=np.int8)
    _check(load().gb_check_mesh_tables(dim, N, vx.shape[0], _dptr(vx), etov.shape[0],
                                       etov.ctypes.data_as(C.POINTER(C.c_int32)),
                                       None if per is None else _dptr(per),
                                       None if tag is None else tag.ctypes.data_as(C.POINTER(C.c_int8))))


def gb_check_batch_layout(dim: int, N: int, precision: int, K, nv, lds_limit: int, cubature_degree: int = 0) -> int:
    """Host-only check of a batched launch class's table layout; returns the
    dynamic LDS bytes of the launch."""
    K = np.ascontiguousarray(K, dtype=np.int64)
    nv = np.ascontiguousarray(nv, dtype=np.int64)
    out = C.c_size_t()
    _check(load().gb_check_batch_layout(dim, N, precision, cubature_degree, K.size,
                                        K.ctypes.data_as(C.POINTER(_i64)), nv.ctypes.data_as(C.POINTER(_i64)),
                                        int(lds_limit), C.byref(out)))
    return out.value


def gb_mesh_destroy(mesh):
    load().gb_mesh_destroy(mesh)


def gb_mesh_sizes(mesh):
    K, Np, NF, Nfp, Nf = _i64(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check(load().gb_mesh_sizes(mesh, C.byref(K), C.byref(Np), C.byref(NF), C.byref(Nfp), C.byref(Nf)))
    return K.value, Np.value, NF.value, Nfp.value, Nf.value


def gb_ref_operator(dim: int, N: int, which: int, cubature_degree: int = 0, capacity: int = 1 << 20):
    buf = np.zeros(capacity)
    n = _i64()
    _check(load().gb_ref_operator(dim, N, cubature_degree, which, _dptr(buf), capacity, C.byref(n)))
    return buf[:n.value].copy()


def gb_mesh_nodes(mesh, dim: int) -> np.ndarray:
    K, Np, *_ = gb_mesh_sizes(mesh)
    out = np.zeros((K, dim, Np))
    _check(load().gb_mesh_nodes(mesh, _dptr(out)))
    return out


def gb_mesh_vertices(mesh, nv: int, dim: int) -> np.ndarray:
    out = np.zeros((nv, dim))
    _check(load().gb_mesh_vertices(mesh, _dptr(out)))
    return out


def gb_set_motion(mesh, kind: int, params=()):
    m = gb_motion()
    m.kind = kind
    for i, v in enumerate(params):
        m.p[i] = float(v)
    _check(load().gb_set_motion(mesh, C.byref(m)))


def gb_set_vertex_velocity(mesh, w):
    """w [4][nv][dim]: vertex velocities at t_n, t_n + dt/2, t_n + dt/2, t_n + dt."""
    w = _f64(w)
    _check(load().gb_set_vertex_velocity(mesh, _dptr(w)))


def make_params(c: float, tau: float, precision: int = GB_FP64, flux_mode: int = GB_FLUX_SPLIT,
                rho0: float = 1.0, cubature_degree: int = 0, q_inf=None, sponge=None) -> gb_params:
    p = gb_params()
    p.c, p.tau, p.precision, p.flux_mode = c, tau, precision, flux_mode
    p.rho0, p.cubature_degree = rho0, cubature_degree
    if q_inf is not None:
        for i, v in enumerate(q_inf):
            p.q_inf[i] = float(v)
    if sponge is not None:
        p.sponge_cx, p.sponge_cy, p.sponge_r0, p.sponge_r1, p.sponge_sigma_max = map(float, sponge)
    return p


def gb_solver_create(mesh, params: gb_params):
    out = _P()
    _check(load().gb_solver_create(mesh, C.byref(params), C.byref(out)))
    return out


def gb_solver_destroy(solver):
    load().gb_solver_destroy(solver)


def gb_solver_footprint(mesh, params: gb_params) -> int:
    n = C.c_size_t()
    _check(load().gb_solver_footprint(mesh, C.byref(params), C.byref(n)))
    return n.value


def gb_state_set(solver, q, t0: float = 0.0):
    q = _f64(q)
    _check(load().gb_state_set(solver, _dptr(q), t0))


def gb_state_set_equilibrium(solver, rho, u, offset=None, t0: float = 0.0):
    """rho [K][Np], u [K][dim][Np] (host FP64); offset [NF] or None."""
    rho, u = _f64(rho), _f64(u)
    off = None if offset is None else _f64(offset)
    _check(load().gb_state_set_equilibrium(solver, _dptr(rho), _dptr(u), None if off is None else _dptr(off), t0))


def gb_equilibrium_moments(dim: int, c: float, rho, u) -> np.ndarray:
    """rho [n], u [dim][n] -> moments [NF][n] (host computation in the library)."""
    rho = _f64(np.atleast_1d(rho))
    u = _f64(np.asarray(u, float).reshape(dim, -1))
    q = np.zeros((6 if dim == 2 else 10, rho.size))
    _check(load().gb_equilibrium_moments(dim, c, rho.size, _dptr(rho), _dptr(u), _dptr(q)))
    return q


def gb_checkpoint_save(solver) -> bytes:
    n = C.c_size_t()
    _check(load().gb_checkpoint_bytes(solver, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(load().gb_checkpoint_save(solver, buf, n.value))
    return buf.raw


def gb_checkpoint_load(solver, data: bytes):
    buf = C.create_string_buffer(data, len(data))
    _check(load().gb_checkpoint_load(solver, buf, len(data)))


def gb_energy(solver, rho_inf: float = 1.0):
    """(E_K, epsilon_1 = -dE_K/dt, domain volume) at the current state."""
    out = np.zeros(3)
    _check(load().gb_energy(solver, rho_inf, _dptr(out)))
    return float(out[0]), float(out[1]), float(out[2])


def gb_energy_noalloc(solver, rho_inf: float = 1.0):
    """gb_energy without device allocation (fixed library scratch)."""
    out = np.zeros(3)
    _check(load().gb_energy_noalloc(solver, rho_inf, _dptr(out)))
    return float(out[0]), float(out[1]), float(out[2])


def gb_wall_force(solver, dim: int):
    """(pressure force [dim], viscous force [dim]) of the fluid on the walls."""
    out = np.zeros(2 * dim)
    _check(load().gb_wall_force(solver, _dptr(out)))
    return out[:dim].copy(), out[dim:].copy()


def gb_state_get(solver, shape=None):
    """(state [K][NF][Np] or None when shape is None, time, steps taken)."""
    q = None if shape is None else np.zeros(shape)
    t = C.c_double()
    step = _i64()
    _check(load().gb_state_get(solver, None if q is None else _dptr(q), C.byref(t), C.byref(step)))
    return q, t.value, step.value


def gb_rhs(solver, q) -> np.ndarray:
    q = _f64(q)
    F = np.zeros_like(q)
    _check(load().gb_rhs(solver, _dptr(q), _dptr(F)))
    return F


def gb_sark_step(solver, dt: float, nsteps: int):
    _check(load().gb_sark_step(solver, dt, nsteps))


def gb_sark_step_graph(solver, dt: float, nsteps: int):
    _check(load().gb_sark_step_graph(solver, dt, nsteps))


def gb_solver_time_stages(solver, enable: bool):
    _check(load().gb_solver_time_stages(solver, 1 if enable else 0))


def gb_solver_stage_time(solver):
    ms = C.c_double()
    n = _i64()
    _check(load().gb_solver_stage_time(solver, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def gb_solver_stage_time_by_kind(solver):
    out = np.zeros(4)
    _check(load().gb_solver_stage_time_by_kind(solver, _dptr(out)))
    return out


def gb_mesh_footprint(mesh) -> int:
    n = C.c_size_t()
    _check(load().gb_mesh_footprint(mesh, C.byref(n)))
    return n.value


def gb_batch_create(ctx, hbm_budget: int):
    out = _P()
    _check(load().gb_batch_create(ctx, int(hbm_budget), C.byref(out)))
    return out


def gb_batch_destroy(batch):
    load().gb_batch_destroy(batch)


def gb_batch_add(batch, solver, dt: float, nsteps: int) -> int:
    """Ticket of the admitted solver; raises GbError with status GB_ERR_BUSY
    when it does not fit the free budget."""
    t = C.c_uint64()
    _check(load().gb_batch_add(batch, solver, dt, nsteps, C.byref(t)))
    return t.value


def gb_batch_run(batch, steps: int):
    _check(load().gb_batch_run(batch, steps))


def gb_batch_poll(batch, capacity: int = 1024) -> list:
    buf = (C.c_uint64 * max(capacity, 1))()
    n = C.c_int()
    _check(load().gb_batch_poll(batch, buf, capacity, C.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


def gb_batch_info(batch):
    a, u, b = C.c_int(), C.c_size_t(), C.c_size_t()
    _check(load().gb_batch_info(batch, C.byref(a), C.byref(u), C.byref(b)))
    return a.value, u.value, b.value


def gb_batch_set_autotune(batch, enable: bool):
    _check(load().gb_batch_set_autotune(batch, 1 if enable else 0))


def gb_batch_set_concurrency(batch, streams: int):
    _check(load().gb_batch_set_concurrency(batch, int(streams)))


def gb_batch_class_count(batch) -> int:
    n = C.c_int()
    _check(load().gb_batch_class_count(batch, C.byref(n)))
    return n.value


def gb_batch_class_info(batch, i: int) -> dict:
    out = (_i64 * 7)()
    _check(load().gb_batch_class_info(batch, i, out))
    return dict(zip(("dim", "N", "precision", "members", "groups", "grid", "solo"), (int(v) for v in out)))


def gb_batch_class_tile(batch, i: int) -> dict:
    out = (_i64 * 3)()
    _check(load().gb_batch_class_tile(batch, i, out))
    return dict(zip(("grid", "waves", "interleave"), (int(v) for v in out)))


def gb_tune_cache_save(path: str):
    _check(load().gb_tune_cache_save(path.encode()))


def gb_tune_cache_load(path: str) -> int:
    n = C.c_int()
    _check(load().gb_tune_cache_load(path.encode(), C.byref(n)))
    return n.value


def gb_tune_cache_clear():
    load().gb_tune_cache_clear()
