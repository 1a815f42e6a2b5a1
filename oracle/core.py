"""ctypes wrapper of the C oracle (``gf_oracle.c``). Test infrastructure only.

Fields are numpy complex128 arrays in the canonical layout
(nt, nz, ny, nx, 4, 3, 3); every function works in place on a C-contiguous
array or returns new numpy objects. dims = (nx, ny, nz, nt).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "gf_oracle_sun.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LANDAU, COULOMB = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction; OpenMP
    shares the sites of a half-sweep among threads)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P, I, L, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double
        lib.oracle_quality.argtypes = [P, P, I, P, P]
        lib.oracle_divergence_field.argtypes = [P, P, I, P]
        lib.oracle_staple.argtypes = [P, P, I, L, P]
        lib.oracle_su2_solve.argtypes = [P, D, P]
        lib.oracle_subgroup_update.argtypes = [P, P, I, L, I, D]
        lib.oracle_site_update.argtypes = [P, P, I, L, D]
        lib.oracle_half_sweep.argtypes = [P, P, I, I, D]
        lib.oracle_half_sweep_order.argtypes = [P, P, I, I, D, P, L]
        lib.oracle_sweep.argtypes = [P, P, I, D]
        lib.oracle_reunit.argtypes = [P, L]
        lib.oracle_fix.argtypes = [P, P, I, D, D, I, I, I, L, P, P, P]
        lib.oracle_fix.restype = I
        lib.oracle_set_threads.argtypes = [I]
        lib.oracle_set_threads.restype = I
        lib.oracle_sun_quality.argtypes = [P, P, I, I, P, P]
        lib.oracle_sun_staple.argtypes = [P, P, I, I, L, P]
        lib.oracle_sun_subgroup_matrix.argtypes = [P, P, I, I, L, I, I, D, P]
        lib.oracle_sun_apply.argtypes = [P, P, I, L, P]
        lib.oracle_sun_subgroup_update.argtypes = [P, P, I, I, L, I, I, D]
        lib.oracle_sun_site_update.argtypes = [P, P, I, I, L, D]
        lib.oracle_sun_half_sweep.argtypes = [P, P, I, I, I, D]
        lib.oracle_sun_sweep.argtypes = [P, P, I, I, D]
        lib.oracle_sun_reunit.argtypes = [P, I, L]
        lib.oracle_sun_det.argtypes = [P, I, L, P]
        lib.oracle_sun_fix.argtypes = [P, P, I, I, D, D, I, I, I, L, P, P, P]
        lib.oracle_sun_fix.restype = I
        _lib = lib
    return _lib


def _dims(dims):
    d = np.asarray([int(x) for x in dims], dtype=np.int32)
    assert d.shape == (4,)
    return d


def _field(U):
    assert isinstance(U, np.ndarray) and U.dtype == np.complex128 and U.flags.c_contiguous
    return U


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def quality(U, dims, gauge=LANDAU):
    """(F, theta) of eqs. (1)-(2)."""
    _field(U)
    d = _dims(dims)
    F, th = ctypes.c_double(), ctypes.c_double()
    load().oracle_quality(_p(U), _p(d), gauge, ctypes.byref(F), ctypes.byref(th))
    return F.value, th.value


def divergence_field(U, dims, gauge=LANDAU):
    """Delta(x) of eq. (3) for every site, shape (V, 3, 3)."""
    _field(U)
    d = _dims(dims)
    V = int(np.prod(d))
    out = np.zeros((V, 3, 3), dtype=np.complex128)
    load().oracle_divergence_field(_p(U), _p(d), gauge, _p(out))
    return out


def staple(U, dims, site, gauge=LANDAU):
    """K(x) of eq. (5) on the current field, shape (3, 3)."""
    _field(U)
    d = _dims(dims)
    out = np.zeros((3, 3), dtype=np.complex128)
    load().oracle_staple(_p(U), _p(d), gauge, int(site), _p(out))
    return out


def su2_solve(b, omega):
    """Overrelaxed local SU(2) solution as a quaternion (4,)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros(4)
    load().oracle_su2_solve(_p(b), float(omega), _p(out))
    return out


def subgroup_update(U, dims, site, sub, omega, gauge=LANDAU):
    load().oracle_subgroup_update(_p(_field(U)), _p(_dims(dims)), gauge, int(site), int(sub), float(omega))


def site_update(U, dims, site, omega, gauge=LANDAU):
    load().oracle_site_update(_p(_field(U)), _p(_dims(dims)), gauge, int(site), float(omega))


def half_sweep(U, dims, parity, omega, gauge=LANDAU):
    load().oracle_half_sweep(_p(_field(U)), _p(_dims(dims)), gauge, int(parity), float(omega))


def half_sweep_order(U, dims, parity, omega, order, gauge=LANDAU):
    order = np.ascontiguousarray(order, dtype=np.int64)
    load().oracle_half_sweep_order(_p(_field(U)), _p(_dims(dims)), gauge, int(parity), float(omega),
                                   _p(order), order.size)


def sweep(U, dims, omega, gauge=LANDAU):
    load().oracle_sweep(_p(_field(U)), _p(_dims(dims)), gauge, float(omega))


def reunit(U):
    _field(U)
    load().oracle_reunit(_p(U), U.size // 9)


def fix(U, dims, omega, eps, max_iter, gauge=LANDAU, reunit_every=20, check_every=1, start_sweep=0):
    """Alg. 1 in place. Returns dict(converged, iters, F, theta)."""
    it = ctypes.c_int()
    F, th = ctypes.c_double(), ctypes.c_double()
    conv = load().oracle_fix(_p(_field(U)), _p(_dims(dims)), gauge, float(omega), float(eps),
                             int(max_iter), int(reunit_every), int(check_every), int(start_sweep),
                             ctypes.byref(it), ctypes.byref(F), ctypes.byref(th))
    return dict(converged=bool(conv), iters=it.value, F=F.value, theta=th.value)


def set_threads(n: int = 0) -> int:
    """Threads shared by the sites of a half-sweep (n <= 0: keep the current
    number). Returns the number in effect."""
    return int(load().oracle_set_threads(int(n)))


def parity_of_sites(dims):
    """Parity (x+y+z+t) mod 2 of every site in canonical order, shape (V,)."""
    nx, ny, nz, nt = (int(x) for x in dims)
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x + y + z + t) & 1).reshape(-1)
