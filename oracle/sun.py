"""ctypes wrapper of the SU(N) oracle (``gf_oracle_sun.c``). Test
infrastructure only.

Fields are numpy complex128 arrays in the canonical layout
(nt, nz, ny, nx, 4, N, N), C-contiguous; functions work in place or return new
numpy objects. dims = (nx, ny, nz, nt); 2 <= N <= 8.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .core import LANDAU, _dims, _p, load

NMAX = 8


def _nc(U):
    assert isinstance(U, np.ndarray) and U.dtype == np.complex128 and U.flags.c_contiguous
    n = U.shape[-1]
    assert U.shape[-2] == n and 2 <= n <= NMAX
    return n


def quality(U, dims, gauge=LANDAU):
    """(F, theta) of eqs. (1)-(2) for SU(N)."""
    n = _nc(U)
    F, th = ctypes.c_double(), ctypes.c_double()
    load().oracle_sun_quality(_p(U), _p(_dims(dims)), n, gauge, ctypes.byref(F), ctypes.byref(th))
    return F.value, th.value


def staple(U, dims, site, gauge=LANDAU):
    """K(x) of eq. (5), shape (N, N)."""
    n = _nc(U)
    out = np.zeros((n, n), dtype=np.complex128)
    load().oracle_sun_staple(_p(U), _p(_dims(dims)), n, gauge, int(site), _p(out))
    return out


def subgroup_matrix(U, dims, site, a, b, omega, gauge=LANDAU):
    """The embedded overrelaxed SU(2) element of subgroup (a, b) at a site, (N, N)."""
    n = _nc(U)
    out = np.zeros((n, n), dtype=np.complex128)
    load().oracle_sun_subgroup_matrix(_p(U), _p(_dims(dims)), n, gauge, int(site), int(a), int(b),
                                      float(omega), _p(out))
    return out


def apply(U, dims, site, G):
    """Rotate the eight links of a site by G (N, N)."""
    n = _nc(U)
    G = np.ascontiguousarray(G, dtype=np.complex128)
    load().oracle_sun_apply(_p(U), _p(_dims(dims)), n, int(site), _p(G))


def subgroup_update(U, dims, site, a, b, omega, gauge=LANDAU):
    load().oracle_sun_subgroup_update(_p(U), _p(_dims(dims)), _nc(U), gauge, int(site), int(a), int(b),
                                      float(omega))


def site_update(U, dims, site, omega, gauge=LANDAU):
    load().oracle_sun_site_update(_p(U), _p(_dims(dims)), _nc(U), gauge, int(site), float(omega))


def half_sweep(U, dims, parity, omega, gauge=LANDAU):
    load().oracle_sun_half_sweep(_p(U), _p(_dims(dims)), _nc(U), gauge, int(parity), float(omega))


def sweep(U, dims, omega, gauge=LANDAU):
    load().oracle_sun_sweep(_p(U), _p(_dims(dims)), _nc(U), gauge, float(omega))


def reunit(U):
    n = _nc(U)
    load().oracle_sun_reunit(_p(U), n, U.size // (n * n))


def det(U):
    """Determinant of every N x N block, flat array."""
    n = _nc(U)
    out = np.zeros(U.size // (n * n), dtype=np.complex128)
    load().oracle_sun_det(_p(U), n, out.size, _p(out))
    return out


def fix(U, dims, omega, eps, max_iter, gauge=LANDAU, reunit_every=20, check_every=1, start_sweep=0):
    """Alg. 1 in place for SU(N). Returns dict(converged, iters, F, theta)."""
    it = ctypes.c_int()
    F, th = ctypes.c_double(), ctypes.c_double()
    conv = load().oracle_sun_fix(_p(U), _p(_dims(dims)), _nc(U), gauge, float(omega), float(eps),
                                 int(max_iter), int(reunit_every), int(check_every), int(start_sweep),
                                 ctypes.byref(it), ctypes.byref(F), ctypes.byref(th))
    return dict(converged=bool(conv), iters=it.value, F=F.value, theta=th.value)
